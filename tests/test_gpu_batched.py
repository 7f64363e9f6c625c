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


def test_batched_errors(gv, collections):
    models = [b[1] for b in collections]
    indexes = [b[2] for b in collections]
    Qs = [b[3] for b in collections]
    with pytest.raises(gv.GleanVecError):
        gv.search_batched(models, indexes, Qs, 10, 100000)  # kappa > n
    with pytest.raises(ValueError):
        gv.search_batched(models[:2], indexes, Qs, 10, 40)
