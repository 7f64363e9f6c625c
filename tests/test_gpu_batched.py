"""Batched search over uneven collections (one captured graph): per collection the
results must equal the single-collection search, on the first call (capture) and
on replays with other device work in between, and after the arguments change."""
import sys

import numpy as np
import pytest

import synth

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


@pytest.fixture(scope="module")
def collections(gv):
    cols = synth.batched_collections(count=7, n_lo=3_000, n_hi=70_000, m_hi=300, dims=(64, 128, 256),
                                     clusters=(1, 4, 8), cfg=41)
    cols[0].m = 0  # an empty batch
    cols[1].m = 1
    built = []
    for c in cols:
        geom = synth.make_geometry(c.cfg, c.D, c.C, "mixture")
        X = torch.from_numpy(synth.database(geom, c.n)).cuda()
        QL = torch.from_numpy(synth.queries(geom, 2000, synth.S_QLEARN)).cuda()
        Q = torch.from_numpy(synth.queries(geom, max(c.m, 1), synth.S_QTEST)[:c.m]).cuda().contiguous()
        model = gv.fit(X, QL, c.d, c.C, seed=c.cfg)
        index = gv.encode(model, X, "bf16", copy_X=True)
        built.append((c, model, index, Q))
    return built


def _eager(gv, built, k, kappa):
    return [gv.search(md, ix, Q, k, kappa) if Q.shape[0] else
            (torch.empty((0, k), dtype=torch.int32, device="cuda"), torch.empty((0, k), device="cuda"))
            for _, md, ix, Q in built]


def _same(a, b):
    for (i1, s1), (i2, s2) in zip(a, b):
        assert torch.equal(i1, i2) and torch.equal(s1, s2)


def test_batched_equals_single_and_replays(gv, collections):
    k, kappa = 10, 40
    _say("[batched] capture")
    ref = _eager(gv, collections, k, kappa)
    models = [b[1] for b in collections]
    indexes = [b[2] for b in collections]
    Qs = [b[3] for b in collections]
    out = gv.search_batched(models, indexes, Qs, k, kappa)
    torch.cuda.synchronize()
    _same(out, ref)
    for rep in range(3):
        _say(f"[batched] replay {rep}")
        for t in out:  # scribble over the outputs so a replay must rewrite them
            t[0].fill_(-7); t[1].fill_(-7.0)
        other = _eager(gv, collections[2:4], k, kappa)  # unrelated device work between replays
        torch.cuda.synchronize()
        out = gv.search_batched(models, indexes, Qs, k, kappa, out=out)
        torch.cuda.synchronize()
        _same(out, ref)
        _same(other, ref[2:4])
    # other arguments: a new capture
    _say("[batched] recapture")
    Qs2 = [Q.flip(0).contiguous() for Q in Qs]
    out2 = gv.search_batched(models, indexes, Qs2, k, kappa)
    torch.cuda.synchronize()
    ref2 = [gv.search(md, ix, Q, k, kappa) if Q.shape[0] else r for md, ix, Q, r in zip(models, indexes, Qs2, ref)]
    _same(out2, ref2)
    gv.batch_release()


def test_batched_collections_match_oracle(gv, collections):
    """Each collection of the batch against the oracle: the batched result equals the
    single search bit for bit, and the single search passes the oracle parity of
    verify_search (every difference from the oracle's encode and search of the same
    rows, with the model's exported projections, proven a near tie)."""
    from helpers import verify_search
    from oracle import gleanvec as G
    k, kappa = 10, 40
    models = [b[1] for b in collections]
    indexes = [b[2] for b in collections]
    Qs = [b[3] for b in collections]
    out = gv.search_batched(models, indexes, Qs, k, kappa)
    torch.cuda.synchronize()
    for j, (c, md, ix, Q) in enumerate(collections):
        if Q.shape[0] == 0:
            continue
        _say(f"[batched] collection {j}: n={c.n} D={c.D} d={c.d} C={c.C} m={c.m}")
        ids, sc = gv.search(md, ix, Q, k, kappa)
        torch.cuda.synchronize()
        assert torch.equal(out[j][0], ids) and torch.equal(out[j][1], sc)
        geom = synth.make_geometry(c.cfg, c.D, c.C, "mixture")
        X = synth.database(geom, c.n)
        mu, A, B = md.export()
        oi = G.encode(mu, B, X, "bf16")
        Qh = Q.cpu().numpy()
        ora = G.search(oi, A, Qh, k, kappa)
        verify_search(gv, md, ix, X, Qh, oi, ora, kappa, k, "bf16", f"collection {j}")
    gv.batch_release()


def test_batched_recaptures_after_an_index_is_replaced(gv, collections):
    """A replay key names handles by generation, not address: destroying an index
    and encoding another (glibc often hands the freed address to the new handle)
    must lead to a new capture whose results equal the single searches."""
    k, kappa = 10, 40
    c, md, ix, Q = collections[3]
    geom = synth.make_geometry(c.cfg, c.D, c.C, "mixture")
    X = torch.from_numpy(synth.database(geom, c.n)).cuda()
    ix1 = gv.encode(md, X, "bf16", copy_X=True)
    out = gv.search_batched([md], [ix1], [Q], k, kappa)
    torch.cuda.synchronize()
    cap0, rep0 = gv.batch_counts()
    out = gv.search_batched([md], [ix1], [Q], k, kappa, out=out)   # same arguments: a replay
    torch.cuda.synchronize()
    cap1, rep1 = gv.batch_counts()
    assert (cap1, rep1) == (cap0, rep0 + 1)
    del ix1
    X2 = X[: c.n // 2].contiguous()                                   # a different index
    ix2 = gv.encode(md, X2, "bf16", copy_X=True)
    out2 = gv.search_batched([md], [ix2], [Q], k, kappa, out=out)
    torch.cuda.synchronize()
    cap2, _ = gv.batch_counts()
    assert cap2 == cap1 + 1
    ids, sc = gv.search(md, ix2, Q, k, kappa)
    torch.cuda.synchronize()
    assert torch.equal(out2[0][0], ids) and torch.equal(out2[0][1], sc)
    gv.batch_release()


def test_batched_errors(gv, collections):
    models = [b[1] for b in collections]
    indexes = [b[2] for b in collections]
    Qs = [b[3] for b in collections]
    with pytest.raises(gv.GleanVecError):
        gv.search_batched(models, indexes, Qs, 10, 100000)  # kappa > n
    with pytest.raises(ValueError):
        gv.search_batched(models[:2], indexes, Qs, 10, 40)


def test_autotune_keeps_results_and_feeds_the_table(gv, collections):
    """The autotuner times launch shapes and stores the fastest for the shape class;
    searches (single and batched) then use it, and their results stay bit-equal to
    the untuned ones (the launch shape never changes a result)."""
    k, kappa = 10, 40
    c, md, ix, Q = collections[4]
    gv.tuning_table_clear()
    ref = gv.search(md, ix, Q, k, kappa)
    r = gv.autotune(md, ix, Q, k, kappa, reps=2)
    _say(f"[autotune] {r}")
    assert r["candidates"] >= 2 and r["ms"] <= r["ms_automatic"] + 1e-9
    assert gv.tuning_lookup("bf16", ix.d_pad, Q.shape[0], ix.rows) == (r["splits"], r["qpw"], r["cap"])
    got = gv.search(md, ix, Q, k, kappa)
    torch.cuda.synchronize()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    models = [b[1] for b in collections]
    indexes = [b[2] for b in collections]
    Qs = [b[3] for b in collections]
    out = gv.search_batched(models, indexes, Qs, k, kappa)
    torch.cuda.synchronize()
    assert torch.equal(out[4][0], ref[0]) and torch.equal(out[4][1], ref[1])
    gv.batch_release()
    gv.tuning_table_clear()


def test_batched_optimistic_seed_repair(gv, collections):
    """kappa = 10 gives the collections of 10^4 rows and more a three-level
    cascade; with the optimistic seed forced to the best sample score, almost
    every query is repaired -- in the persistent batched executor as in the single
    searches -- and the results equal the automatic ones."""
    k, kappa = 10, 10
    models = [md for _, md, _, _ in collections]
    indexes = [ix for _, _, ix, _ in collections]
    Qs = [Q for _, _, _, Q in collections]
    ref = _eager(gv, collections, k, kappa)
    try:
        gv.search_optimism(1)
        forced = _eager(gv, collections, k, kappa)
        out = gv.search_batched(models, indexes, Qs, k, kappa)
        torch.cuda.synchronize()
        _same(forced, ref)
        _same(out, ref)
    finally:
        gv.search_optimism(0)
        gv.batch_release()
