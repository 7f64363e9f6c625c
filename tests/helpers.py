"""Shared test helpers: seeded problems and the comparison rules of the parity
tests (tolerances derived from the arithmetic, near-tie handling for top-k)."""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import formats
from oracle import gleanvec as G

U32 = 2.0 ** -24


@functools.lru_cache(maxsize=None)
def problem(cfg: int, D: int, J: int, n: int, m_learn: int, m: int, law: str = "mixture"):
    """Seeded database, learn queries and test queries (FP32 numpy)."""
    geom = synth.make_geometry(cfg, D, J, law)
    X = synth.database(geom, n)
    QL = synth.queries(geom, m_learn, synth.S_QLEARN)
    Q = synth.queries(geom, m, synth.S_QTEST)
    return X, QL, Q


@functools.lru_cache(maxsize=None)
def oracle_model(cfg, D, J, n, m_learn, d, C, seed, law="mixture"):
    X, QL, _ = problem(cfg, D, J, n, m_learn, 1, law)
    return G.fit(X, QL, d, C, seed)


def decode_stored(fmt: str, bits: np.ndarray) -> np.ndarray:
    if fmt == "fp32":
        return bits.view(np.float32).astype(np.float64)
    return formats.decode(fmt, bits)


def reduced_score_tolerance(out, index, K: int) -> np.ndarray:
    """|s_gpu - s_exact| bound for FP32 accumulation of K exact products:
    (K + 2) * 2^-24 * s_c * t * sum_j |q^_j x^_j| (+ one rounding of the result)."""
    m = out["qh"].shape[0]
    n = index.xq.shape[0]
    tol = np.empty((m, n))
    for c in range(index.offsets.shape[0] - 1):
        a, b = index.offsets[c], index.offsets[c + 1]
        if a == b:
            continue
        ds = out["qh"].shape[2]  # leading coordinates scored (all of them unless flexible d)
        absdot = np.abs(out["qh"][:, c, :]) @ np.abs(index.xq[a:b, :ds]).T
        tol[:, a:b] = (K + 2) * U32 * absdot * (index.scale[c] * out["t"][:, c])[:, None]
    return tol + np.abs(out["scores"]) * U32


def _oracle_topk(scores_by_id, kappa):
    """The oracle's top-kappa of one score vector indexed by id; the oracle's own
    ordering runs on every element that can reach the kappa-th score (ties included),
    which gives the same result as running it on all of them."""
    n = scores_by_id.shape[0]
    if n > 4 * kappa:
        kth = np.partition(scores_by_id, n - kappa)[n - kappa]
        sub = np.nonzero(scores_by_id >= kth)[0]
    else:
        sub = np.arange(n)
    return G.topk(scores_by_id[sub], sub, kappa)


def check_topk_sets(gpu_ids, gpu_scores, ora_scores_by_id, tol_by_id, kappa, what=""):
    """GPU and oracle top-kappa sets may differ only in elements whose oracle score is
    within tolerance of the oracle's kappa-th score; GPU scores must match the
    oracle's within tolerance and be ordered (desc, ties by id)."""
    ora_ids, ora_sc = _oracle_topk(ora_scores_by_id, kappa)
    kth = ora_sc[-1]
    kth_tol = tol_by_id[ora_ids[-1]]
    g = set(gpu_ids.tolist())
    o = set(ora_ids.tolist())
    assert len(g) == kappa, f"{what}: duplicate or missing ids"
    for i in g ^ o:
        assert abs(ora_scores_by_id[i] - kth) <= tol_by_id[i] + kth_tol, \
            f"{what}: id {i} score {ora_scores_by_id[i]} vs kappa-th {kth}"
    err = np.abs(gpu_scores.astype(np.float64) - ora_scores_by_id[gpu_ids])
    assert np.all(err <= tol_by_id[gpu_ids]), f"{what}: max score error {err.max()}"
    s = gpu_scores
    order_ok = np.all((s[:-1] > s[1:]) | ((s[:-1] == s[1:]) & (gpu_ids[:-1] < gpu_ids[1:])))
    assert order_ok, f"{what}: candidate list not ordered"
    return len(g ^ o) // 2


def exact_scores(X, q, ids):
    """Exact <q, x_i> in FP64 of the FP32 values, and the bound on the difference of
    any two FP64 summation orders of the same exact products: D * 2^-53 * sum |q_j x_ij|."""
    Xi = np.asarray(X[ids], np.float64)
    q64 = np.asarray(q, np.float64)
    ex = Xi @ q64
    tol = (Xi.shape[1] + 2) * 2.0 ** -53 * (np.abs(Xi) @ np.abs(q64)) + 1e-300
    return ex, tol


def check_final_topk(gpu_ids, gpu_cand, final_scores, final_tol, k, what=""):
    """Stage S4 on the GPU's own candidates: the GPU's final ids must be the k best of
    its candidate list by the rerank score (score desc, id asc), except where two
    candidates lie within the arithmetic tolerance of the k-th score.

    final_scores, final_tol: the oracle-side rerank score of every candidate in
    gpu_cand (same order) and the bound on its difference from the GPU's arithmetic.
    Together with check_topk_sets on gpu_cand, every difference between the GPU's
    final top-k and the oracle's is shown to come from near ties: at the kappa-th
    reduced score (the candidate sets) or at the k-th rerank score (here)."""
    cand = np.asarray(gpu_cand, np.int64)
    keep = cand >= 0
    cand, sc, tl = cand[keep], np.asarray(final_scores)[keep], np.asarray(final_tol)[keep]
    want_ids, want_sc = G.topk(sc, cand, k)
    got = np.asarray(gpu_ids, np.int64)
    assert len(set(got.tolist())) == got.shape[0] == min(k, cand.shape[0]), f"{what}: duplicate or missing ids"
    by = dict(zip(cand.tolist(), zip(sc.tolist(), tl.tolist())))
    for i in got.tolist():
        assert i in by, f"{what}: final id {i} is not a candidate"
    kth_s, kth_t = by[int(want_ids[-1])]
    diff = set(got.tolist()) ^ set(want_ids.tolist())
    for i in diff:
        s, t = by[i]
        assert abs(s - kth_s) <= t + kth_t, f"{what}: final id {i} ({s}) differs away from the k-th score {kth_s}"
    # the GPU's order follows its scores: check it on the oracle-side scores up to tolerance
    for a, b in zip(got[:-1].tolist(), got[1:].tolist()):
        (sa, ta), (sb, tb) = by[a], by[b]
        assert sa >= sb - ta - tb, f"{what}: final list not ordered ({a}: {sa}, {b}: {sb})"
    return len(diff) // 2


def verify_search(gv, model, idx, X, Q, oi, out, kappa, k, fmt, what):
    """End-to-end search against the oracle with every difference proven a near tie:
    the search equals the composition of its stages bit for bit; the GPU's
    candidates pass check_topk_sets against the oracle's reduced scores; its final
    ids are the rerank top-k of its own candidates (check_final_topk); its scores
    are fl32 of the exact inner products.  Returns (queries equal to the oracle's
    final list, GPU ids)."""
    import torch
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to("cuda")
    ids, sc = gv.search(model, idx, Qd, k, kappa)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    cid, csc = gv.score_topk(idx, qhat, t, kappa)
    rid, rsc = gv.rerank(idx, Qd, cid, k)
    torch.cuda.synchronize()
    assert torch.equal(ids, rid) and torch.equal(sc, rsc), f"{what}: search differs from its stages"
    ids = ids.cpu().numpy(); sc = sc.cpu().numpy(); cid = cid.cpu().numpy(); csc = csc.cpu().numpy()
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    agree = 0
    for qi in range(Q.shape[0]):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"{what} q{qi}")
        ex, tl = exact_scores(X, Q[qi], cid[qi])
        check_final_topk(ids[qi], cid[qi], ex, tl, k, f"{what} q{qi}")
        exi, _ = exact_scores(X, Q[qi], ids[qi])
        assert np.array_equal(sc[qi], exi.astype(np.float32)) or \
            np.allclose(sc[qi], exi.astype(np.float32), rtol=2 ** -23, atol=0)
        assert np.all(np.diff(sc[qi]) <= 0)
        agree += ids[qi].tolist() == out["ids"][qi].tolist()
    return agree, ids
