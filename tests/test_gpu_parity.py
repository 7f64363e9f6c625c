"""Parity of the HIP path with the FP64 oracle, stage by stage, through the C ABI.

Sizes are small enough for the oracle to finish in seconds but span several
tiles, several clusters, ragged segment tails and every launch regime of the
scoring kernel (queries shared across wavefronts or split across them)."""
import sys

import numpy as np
import pytest

from helpers import (U32, check_topk_sets, decode_stored, oracle_model, problem,
                     reduced_score_tolerance, verify_search)
from oracle import formats
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


# (cfg, D, J, n, m_learn, d, C, m, kappa)
CASES = {
    "d16-C4": (101, 64, 4, 20_000, 2_000, 16, 4, 37, 50),
    "d40-C8": (102, 128, 8, 30_000, 3_000, 40, 8, 70, 100),
    "d160-C8": (103, 256, 8, 24_000, 4_000, 160, 8, 65, 200),
    # large enough for the threshold cascade: dense sample, pilot scan, full scan
    "n300k": (106, 64, 4, 300_000, 2_000, 32, 4, 40, 50),
    # the benchmark's reduced length (d = 160) and kappa = 200 on a database with two
    # cascade levels below the full scan (every 256th tile dense, every 16th filtered)
    "d160-n420k": (107, 256, 8, 420_000, 4_000, 160, 8, 64, 200),
    # d = 160 with three levels at small batches (every 4096th tile dense, every
    # 64th filtered, then the full scan) and four at large ones (4096, 256, 16, 1):
    # the sampled-level kernels the benchmark launches at m = 1, 64 and 4096
    "d160-n700k": (110, 256, 8, 700_000, 4_000, 160, 8, 64, 20),
    # the longest reduced rows (12 and 16 KiB tiles in 16-bit storage)
    "d192-C8": (108, 384, 8, 24_000, 4_000, 192, 8, 130, 200),
    "d256-C8": (109, 512, 8, 24_000, 4_000, 256, 8, 130, 200),
}


# ----------------------------------------------------------------------------- fit

@pytest.mark.parametrize("case", ["d16-C4", "d40-C8"])
def test_fit_matches_oracle(gv, case):
    cfg, D, J, n, ml, d, C, m, kappa = CASES[case]
    _say(f"[fit] {case}")
    X, QL, _ = problem(cfg, D, J, n, ml, 1)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.fit(dev(X), dev(QL), d, C, seed=7)
    st = model.stats()
    mu, A, B = model.export()
    assert st["iters"] == om.kmeans_iters
    assert np.allclose(mu, om.mu, atol=1e-10)
    assert np.array_equal(st["counts"], om.counts)
    assert np.allclose(st["KQ"], om.KQ, rtol=0, atol=1e-12 * np.abs(om.KQ).max())
    assert np.allclose(st["KX"], om.KX, rtol=0, atol=1e-12 * np.abs(om.KX).max())
    assert np.allclose(st["lam_Q"], om.lam_Q, rtol=0, atol=1e-11 * om.lam_Q[0])
    for c in range(C):
        lam = om.lam_c[c]
        assert np.allclose(st["lam_c"][c], lam, rtol=0, atol=1e-10 * lam[0])
        M_gpu = A[c].T @ B[c]
        M_ora = om.A[c].T @ om.B[c]
        assert np.abs(M_gpu - M_ora).max() <= 1e-7 * np.abs(M_ora).max()
        # same canonical signs, so the rows agree too
        assert np.abs(A[c] - om.A[c]).max() <= 1e-6 * np.abs(om.A[c]).max()
        assert np.abs(B[c] - om.B[c]).max() <= 1e-6 * np.abs(om.B[c]).max()


def test_fit_kmeans_subsample_and_fallback(gv):
    """k-means on a SplitMix64 sample smaller than the learn set, and a cluster count
    high enough that some clusters fall back to the pooled projection."""
    cfg, D, J, n, ml = 104, 32, 3, 6_000, 800
    d, C = 24, 12
    _say("[fit] subsample")
    X, QL, _ = problem(cfg, D, J, n, ml, 1)
    om = G.fit(X, QL, d, C, 99, kmeans_sample=1500, max_iter=8)
    model = gv.fit(dev(X), dev(QL), d, C, seed=99, kmeans_sample=1500, max_iter=8)
    st = model.stats()
    mu, A, B = model.export()
    assert st["iters"] == om.kmeans_iters
    assert np.allclose(mu, om.mu, atol=1e-9)
    assert np.array_equal(st["counts"], om.counts)
    assert np.array_equal(st["fallback"], om.fallback)
    for c in range(C):
        assert np.abs(A[c].T @ B[c] - om.A[c].T @ om.B[c]).max() <= 1e-6


def test_fit_sphering_identities_on_gpu(gv):
    """Pins of the paper on the device fit itself: whitened sphered queries (T2) and
    exact inner products at d = D (T4)."""
    cfg, D, J, n, ml = 105, 24, 1, 3_000, 2_000
    _say("[fit] identities")
    X, QL, _ = problem(cfg, D, J, n, ml, 1)
    model = gv.fit(dev(X), dev(QL), D, 1, seed=1)
    _, A, B = model.export()
    assert np.allclose(A[0].T @ B[0], np.eye(D), atol=1e-9)
    model = gv.fit(dev(X), dev(QL), 10, 1, seed=1)
    _, A, B = model.export()
    Z = QL.astype(np.float64) @ A[0].T
    assert np.allclose(Z.T @ Z / ml, np.eye(10), atol=1e-9)


# ----------------------------------------------------------------------------- encode

@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("case", ["d16-C4", "d40-C8", "d160-C8"])
def test_encode_matches_oracle(gv, case, fmt):
    cfg, D, J, n, ml, d, C, m, kappa = CASES[case]
    _say(f"[encode] {case} {fmt}")
    X, QL, _ = problem(cfg, D, J, n, ml, 1)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    oi = G.encode(om.mu, om.B, X, fmt)
    model = gv.model_import(om.mu, om.A, om.B)
    Xd = dev(X)
    idx = gv.encode(model, Xd, fmt)
    ex = idx.export()
    # tags: FP64 arg-max; a differing tag must be a near tie of the two best landmarks
    dots = X.astype(np.float64) @ om.mu.T
    diff = np.nonzero(ex["tags"] != oi.tags)[0]
    for i in diff:
        top = np.sort(dots[i])[::-1]
        assert top[0] - top[1] <= 1e-13 * np.abs(X[i]).sum()
    assert diff.size <= 2
    if diff.size:
        pytest.skip("near-tie tag: grouping differs legitimately")
    assert np.array_equal(ex["offsets"], oi.offsets)
    assert np.array_equal(ex["ids"], oi.ids)
    s_ref = oi.scale.astype(np.float32)
    assert np.array_equal(ex["scale"], s_ref)
    got = decode_stored(fmt, ex["xlow"])
    assert np.all(got[:, d:] == 0)
    got = got[:, :d]
    same = got == oi.xq
    # v = fl32(B_c x) with FP64 accumulation: at most rare one-ulp differences from
    # the summation order, hence rare one-step differences after rounding
    assert same.mean() > 0.9999
    if not same.all():
        bad = ~same
        step = np.abs(got[bad] - oi.xq[bad])
        ulp = np.abs(oi.xq[bad]) * (2.0 ** -3 if fmt == "fp8" else 2.0 ** -7 if fmt == "bf16" else 2.0 ** -10 if fmt == "fp16" else 2.0 ** -23)
        assert np.all(step <= ulp * 1.0001 + 1e-30)


# ----------------------------------------------------------------------------- S1

@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("m", [5, 70])
def test_project_matches_oracle(gv, fmt, m):
    cfg, D, J, n, ml, d, C, _, kappa = CASES["d40-C8"]
    _say(f"[project] {fmt} m{m}")
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    qc, t, qhat = gv.project(model, fmt, dev(Q))
    torch.cuda.synchronize()
    ref_qc, ref_t, ref_qh = G.project_queries(om.A, Q, fmt)
    qc = qc.cpu().numpy().astype(np.float64)
    assert np.all(qc[:, :, d:] == 0)
    same = qc[:, :, :d] == ref_qc
    assert same.mean() > 0.9999
    assert np.allclose(qc[:, :, :d], ref_qc, rtol=2 ** -23, atol=0)
    t = t.cpu().numpy().astype(np.float64)
    vf = G.VIEW_FORMAT[fmt]  # FP8 storage meets FP16 views
    bits = qhat.cpu().numpy()
    bits = bits.view(np.uint32) if vf == "fp32" else bits.view(np.uint16)
    got = decode_stored(vf, bits)
    assert np.all(got[:, :, d:] == 0)
    got = got[:, :, :d]
    # each device step is exact given the device's own q_c: t from its amax, q^ the
    # nearest view value of q_c / t (so a differing code can only come from a q_c that
    # differs by one FP32 ulp, and then differs by at most one step of the view grid)
    assert np.array_equal(t, formats.pow2_scale(vf, np.abs(qc[:, :, :d]).max(axis=2)))
    assert np.array_equal(got, formats.round_to(vf, qc[:, :, :d] / t[:, :, None]))
    assert np.array_equal(t, ref_t) or np.mean(t == ref_t) > 0.999
    bad = got != ref_qh
    assert bad.mean() <= 1e-4
    if bad.any():
        assert np.all(qc[:, :, :d][bad] != ref_qc[bad])     # only where q_c differs
        tb = np.broadcast_to(t[:, :, None], got.shape)[bad]
        grid = {"fp32": 23, "fp16": 10, "bf16": 7}[vf]
        step = np.ldexp(1.0, np.frexp(np.maximum(np.abs(got[bad]), np.abs(ref_qh[bad])))[1] - 1 - grid)
        assert np.all(np.abs(got[bad] - ref_qh[bad]) <= step), "a view code differs by more than one step"
        assert np.all(tb > 0)


def test_project_large_batch_matches_oracle(gv):
    """S1 for a large batch (6600 queries x 8 clusters x 160 rows, a grid of many
    FP64 matrix-core tiles): q_c equals the oracle's fl32 of the FP64 product
    wherever FP64 summation order cannot flip the rounding, and is within one
    FP32 ulp everywhere."""
    cfg, D, J, n, ml, d, C, _, kappa = CASES["d160-C8"]
    m = 6600
    _say(f"[project large batch] m{m}")
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    qc, t, qhat = gv.project(model, "fp16", dev(Q))
    torch.cuda.synchronize()
    ref_qc, ref_t, ref_qh = G.project_queries(om.A, Q, "fp16")
    qc = qc.cpu().numpy().astype(np.float64)
    assert np.all(qc[:, :, d:] == 0)
    assert (qc[:, :, :d] == ref_qc).mean() > 0.9999
    assert np.allclose(qc[:, :, :d], ref_qc, rtol=2 ** -23, atol=0)


@pytest.mark.parametrize("C,d,D,m", [(3, 24, 100, 17), (3, 24, 100, 300), (4, 160, 768, 64), (2, 40, 64, 33)])
def test_project_mid_batches_match_oracle(gv, C, d, D, m):
    """S1 for batches between the few-query path and the tiled GEMM (16 queries x
    16 rows per workgroup, D cut into 16 runs): ragged query and row tiles, and
    D not a multiple of 16 (the last runs are partly or wholly past D).  q_c is
    the oracle's fl32 of the FP64 product wherever FP64 summation order cannot
    flip the rounding, and within one FP32 ulp everywhere; the padding is zero."""
    _say(f"[project mid] C{C} d{d} D{D} m{m}")
    rng = np.random.default_rng(1000 + m + D)
    mu = rng.standard_normal((C, D))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    A = rng.standard_normal((C, d, D)) / np.sqrt(D)
    B = rng.standard_normal((C, d, D)) / np.sqrt(D)
    Q = rng.standard_normal((m, D)).astype(np.float32)
    model = gv.model_import(mu, A, B)
    qc, t, qhat = gv.project(model, "fp16", dev(Q))
    torch.cuda.synchronize()
    ref_qc, ref_t, ref_qh = G.project_queries(A, Q, "fp16")
    qc = qc.cpu().numpy().astype(np.float64)
    assert np.all(qc[:, :, d:] == 0)
    assert (qc[:, :, :d] == ref_qc).mean() > 0.9999
    assert np.allclose(qc[:, :, :d], ref_qc, rtol=2 ** -23, atol=0)


# ----------------------------------------------------------------------------- S2 + S3 (+ S4)

REGIMES = [
    # (case, m, label): m <= 32 one shared block of 32 queries; m <= 64 two blocks;
    # m > 64 four wavefronts with 128 queries each
    ("d16-C4", 1, "m1"),
    ("d16-C4", 37, "m37"),
    ("d40-C8", 64, "m64"),
    ("d40-C8", 70, "m70"),
    ("d160-C8", 65, "m65"),
    ("d160-C8", 600, "m600"),
    ("n300k", 1, "m1"),
    ("n300k", 40, "m40"),
    ("n300k", 130, "m130"),
    ("d160-n420k", 1, "m1"),
    ("d160-n420k", 40, "m40"),
    ("d160-n420k", 64, "m64"),
    ("d160-n700k", 1, "m1"),
    ("d160-n700k", 40, "m40"),
    ("d160-n700k", 64, "m64"),
    ("d160-n700k", 300, "m300"),
]


def _search_setup(gv, case, fmt, m):
    cfg, D, J, n, ml, d, C, _, kappa = CASES[case]
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    oi = G.encode(om.mu, om.B, X, fmt)
    model = gv.model_import(om.mu, om.A, om.B)
    Xd = dev(X)
    idx = gv.encode(model, Xd, fmt)
    return X, Q, om, oi, model, idx, Xd, kappa


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("case,m,label", REGIMES)
def test_score_topk_matches_oracle(gv, case, m, label, fmt):
    _say(f"[score_topk] {case} {label} {fmt}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, case, fmt, m)
    if not np.array_equal(idx.export()["tags"], oi.tags):
        pytest.skip("near-tie tag")
    out = G.search(oi, om.A, Q, 10, kappa)
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    cid, csc = gv.score_topk(idx, qhat, t, kappa)
    torch.cuda.synchronize()
    cid = cid.cpu().numpy()
    csc = csc.cpu().numpy()
    dp = idx.d_pad
    tol = reduced_score_tolerance(out, oi, dp)
    n = X.shape[0]
    flips = 0
    for qi in range(m):
        by_id = np.empty(n)
        by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n)
        tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(2, m // 20)


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("case,m", [("d16-C4", 37), ("d160-C8", 65)])
def test_search_end_to_end(gv, case, m, fmt):
    _say(f"[search] {case} m{m} {fmt}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, case, fmt, m)
    if not np.array_equal(idx.export()["tags"], oi.tags):
        pytest.skip("near-tie tag")
    out = G.search(oi, om.A, Q, 10, kappa)
    agree, ids = verify_search(gv, model, idx, X, Q, oi, out, kappa, 10, fmt, f"{case} {fmt}")
    _say(f"[search] {agree}/{m} queries equal the oracle's final list, the rest proven near ties")
    gt, _ = G.exact_topk(X, Q, 10)
    r_gpu = G.recall(ids, gt)
    r_ora = G.recall(out["ids"], gt)
    assert abs(r_gpu - r_ora) <= 0.02


def test_rerank_matches_oracle(gv):
    cfg, D, J, n, ml, d, C, m, kappa = CASES["d40-C8"]
    _say("[rerank]")
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    Xd = dev(X)
    idx = gv.encode(model, Xd, "fp16")
    rng = np.random.default_rng(3)
    cand = np.stack([rng.choice(n, kappa, replace=False) for _ in range(m)]).astype(np.int32)
    ids, sc = gv.rerank(idx, dev(Q), dev(cand), 10)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy(); sc = sc.cpu().numpy()
    for qi in range(m):
        ex = X[cand[qi]].astype(np.float64) @ Q[qi].astype(np.float64)
        want_ids, want_sc = G.topk(ex, cand[qi].astype(np.int64), 10)
        assert ids[qi].tolist() == want_ids.tolist()
        assert np.array_equal(sc[qi], want_sc.astype(np.float32))


# ----------------------------------------------------------------------------- edges

def test_edge_cases(gv):
    _say("[edges]")
    cfg, D, J, n, ml, d, C, m, kappa = CASES["d16-C4"]
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    # tiny database: kappa == n, k == kappa, clusters of a handful of rows
    Xs = X[:40]
    idx = gv.encode(model, dev(Xs), "fp16")
    ids, sc = gv.search(model, idx, dev(Q[:5]), 40, 40)
    torch.cuda.synchronize()
    ex = Q[:5].astype(np.float64) @ Xs.astype(np.float64).T
    for qi in range(5):
        want, _ = G.topk(ex[qi], np.arange(40), 40)
        assert ids[qi].cpu().numpy().tolist() == want.tolist()
    # m == 0 is a no-op
    e_ids, _ = gv.search(model, idx, dev(Q[:0]), 5, 10)
    assert e_ids.shape == (0, 5)
    # an empty cluster: a landmark no row is closest to
    away = -om.mu.sum(0)
    mu = np.vstack([om.mu, away / np.linalg.norm(away)])
    A = np.concatenate([om.A, om.A[:1]]); B = np.concatenate([om.B, om.B[:1]])
    m2 = gv.model_import(mu, A, B)
    idx2 = gv.encode(m2, dev(X), "fp8")
    ex2 = idx2.export()
    oi2 = G.encode(mu, B, X, "fp8")
    assert np.array_equal(ex2["offsets"], oi2.offsets)
    out2 = G.search(oi2, A, Q[:3], 10, 50)
    verify_search(gv, m2, idx2, X, Q[:3], oi2, out2, 50, 10, "fp8", "empty cluster")
    # invalid arguments come back as errors, not crashes
    with pytest.raises(gv.GleanVecError):
        gv.search(model, idx, dev(Q[:2]), 10, 41)        # kappa > n
    with pytest.raises(gv.GleanVecError):
        gv.search(model, idx, dev(Q[:2]), 20, 10)        # k > kappa
    bad = X[:50].copy(); bad[3, 2] = np.inf
    with pytest.raises(gv.GleanVecError):
        gv.encode(model, dev(bad), "fp16")


def test_deterministic_repeat(gv):
    _say("[determinism]")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, "d160-C8", "fp8", 300)
    Qd = dev(Q)
    a1, s1 = gv.search(model, idx, Qd, 10, kappa)
    a2, s2 = gv.search(model, idx, Qd, 10, kappa)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(s1, s2)
    _, t, qhat = gv.project(model, "fp8", Qd, want_qc=False)
    c1, d1 = gv.score_topk(idx, qhat, t, kappa)
    gv.search_tuning(splits=24, qpw=0)
    try:
        c2, d2 = gv.score_topk(idx, qhat, t, kappa)
    finally:
        gv.search_tuning(0, 0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(d1, d2)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8"])
def test_long_lists_tile_ring(gv, fmt):
    """Many queries (four query blocks of a workgroup share each row tile through
    an LDS ring) and one row range per query at the default list capacity: every
    list collects all the survivors of its query and is compacted many times from
    lengths at the limit of the wavefront's LDS staging.  Two of the four
    wavefronts hold no queries (padding blocks) and still take part in the ring."""
    m = 130
    _say(f"[long lists] {fmt} m{m}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, "d160-C8", fmt, m)
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    c1, d1 = gv.score_topk(idx, qhat, t, kappa)
    gv.search_tuning(splits=1, qpw=0, cap=0)
    try:
        c2, d2 = gv.score_topk(idx, qhat, t, kappa)
    finally:
        gv.search_tuning(0, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(d1, d2)
    out = G.search(oi, om.A, Q, 10, kappa)
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    c2 = c2.cpu().numpy(); d2 = d2.cpu().numpy()
    flips = 0
    for qi in range(m):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(c2[qi], d2[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(1, m // 50)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8"])
@pytest.mark.parametrize("case", ["d192-C8", "d256-C8"])
def test_tile_ring_longest_rows(gv, case, fmt):
    """Reduced lengths 192 and 256 with many queries: the workgroup-shared tile
    ring at two workgroups per CU (a ring of three 12 KiB tiles; three 16 KiB tiles
    beside a 768-key compaction staging).  Candidates match the oracle, at the
    automatic shape and with one row range per query (long lists compacted at the
    staging's limit), and both shapes give the same lists."""
    _, _, _, _, _, _, _, m, _ = CASES[case]
    _say(f"[ring] {case} {fmt} m{m}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, case, fmt, m)
    if not np.array_equal(idx.export()["tags"], oi.tags):
        pytest.skip("near-tie tag")
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    c1, d1 = gv.score_topk(idx, qhat, t, kappa)
    gv.search_tuning(splits=1, qpw=0, cap=0)
    try:
        c2, d2 = gv.score_topk(idx, qhat, t, kappa)
    finally:
        gv.search_tuning(0, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(d1, d2)
    out = G.search(oi, om.A, Q, 10, kappa)
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    c1 = c1.cpu().numpy(); d1 = d1.cpu().numpy()
    flips = 0
    for qi in range(m):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(c1[qi], d1[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(2, m // 20)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_kappa_beyond_ring_staging(gv, fmt):
    """kappa = 1000 with 130 queries: more than a tile-ring workgroup's compaction
    staging can keep, so the plan takes shared query blocks whose wavefronts stage
    whole lists.  The candidates match the oracle and the end-to-end search is
    proven against it."""
    m, kappa = 130, 1000
    _say(f"[kappa {kappa}] {fmt} m{m}")
    X, Q, om, oi, model, idx, Xd, _ = _search_setup(gv, "d160-C8", fmt, m)
    if not np.array_equal(idx.export()["tags"], oi.tags):
        pytest.skip("near-tie tag")
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    cid, csc = gv.score_topk(idx, qhat, t, kappa)
    torch.cuda.synchronize()
    out = G.search(oi, om.A, Q, 10, kappa)
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    cid = cid.cpu().numpy(); csc = csc.cpu().numpy()
    flips = 0
    for qi in range(m):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(2, m // 20)
    verify_search(gv, model, idx, X, Q, oi, out, kappa, 10, fmt, f"kappa {kappa} {fmt}")


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case,m", [("n300k", 130), ("d160-n420k", 64), ("d160-n700k", 64), ("d160-n700k", 300)])
def test_optimistic_seed_and_repair(gv, case, m, fmt):
    """The full scan starts from an optimistic seed (a higher-ranked score of the
    last sample level) and a repair pass rescans every query that kept fewer than
    kappa keys.  Forcing the repair for almost every query (rank 1), the
    automatic rank, and the exact kappa-th best of the sample (rank -1) give the
    same candidates bit for bit, in the stage call and in the end-to-end search;
    the candidates match the oracle."""
    _say(f"[optimism] {case} m{m} {fmt}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, case, fmt, m)
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    got = {}
    try:
        for rank in (0, 1, -1):
            gv.search_optimism(rank)
            got[rank] = (gv.score_topk(idx, qhat, t, kappa), gv.search(model, idx, Qd, 10, kappa))
    finally:
        gv.search_optimism(0)
    torch.cuda.synchronize()
    for rank in (1, -1):
        for a, b in zip(got[rank], got[0]):
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), f"rank {rank}"
    if not np.array_equal(idx.export()["tags"], oi.tags):
        return  # a near-tie tag: the oracle comparison is covered by the other tests
    out = G.search(oi, om.A, Q, 10, kappa)
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    cid = got[0][0][0].cpu().numpy(); csc = got[0][0][1].cpu().numpy()
    flips = 0
    for qi in range(m):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(2, m // 20)


@pytest.mark.parametrize("fmt", ["fp16", "fp8"])
@pytest.mark.parametrize("m", [20, 65])
def test_compaction_path(gv, fmt, m):
    """Few row ranges and a small candidate cap force many in-loop compactions
    (wavefront radix select + threshold raise); the result must not change."""
    _say(f"[compaction] {fmt} m{m}")
    X, Q, om, oi, model, idx, Xd, kappa = _search_setup(gv, "d160-C8", fmt, m)
    Qd = dev(Q)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    c1, d1 = gv.score_topk(idx, qhat, t, kappa)
    gv.search_tuning(splits=4, qpw=0, cap=640)
    try:
        c2, d2 = gv.score_topk(idx, qhat, t, kappa)
    finally:
        gv.search_tuning(0, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(d1, d2)
    out = G.search(oi, om.A, Q, 10, kappa)
    tol = reduced_score_tolerance(out, oi, idx.d_pad)
    n = X.shape[0]
    c2 = c2.cpu().numpy(); d2 = d2.cpu().numpy()
    for qi in range(m):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        check_topk_sets(c2[qi], d2[qi], by_id, tol_id, kappa, f"q{qi}")
