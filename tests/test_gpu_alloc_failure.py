"""Out-of-memory paths: every device allocation the library makes in encode, a
search, a batched search and a fit is made to fail in turn
(gv_debug_fail_alloc); each such call must return GV_ENOMEM without side
effects, and the same call made afterwards must succeed with the results of an
undisturbed run."""
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
def problem(gv):
    geom = synth.make_geometry(61, 96, 4, "mixture")
    X = torch.from_numpy(synth.database(geom, 40_000)).cuda()
    QL = torch.from_numpy(synth.queries(geom, 2_000, synth.S_QLEARN)).cuda()
    Q = torch.from_numpy(synth.queries(geom, 90, synth.S_QTEST)).cuda()
    model = gv.fit(X, QL, 24, 4, seed=3)
    return X, QL, Q, model


def _sweep(gv, call, what, limit=200):
    """Fail the 1st, 2nd, ... allocation of `call` until it runs through; every
    failing run raises GV_ENOMEM.  Returns the number of allocations seen."""
    for after in range(limit):
        gv.debug_fail_alloc(after)
        try:
            call()
        except gv.GleanVecError as e:
            assert e.status == -2, f"{what}: allocation {after} failed with {e}"
            continue
        finally:
            pending = gv.debug_allocs_pending()
            gv.debug_fail_alloc(-1)
        assert pending >= 0, f"{what}: the forced failure at allocation {after} went unreported"
        _say(f"[alloc] {what}: {after} allocations, each failure reported as GV_ENOMEM")
        return after
    raise AssertionError(f"{what}: more than {limit} allocations")


def test_encode_and_search_survive_each_allocation_failure(gv, problem):
    X, QL, Q, model = problem
    ref_idx = gv.encode(model, X, "fp16")
    ref = gv.search(model, ref_idx, Q, 10, 60)
    torch.cuda.synchronize()
    n_enc = _sweep(gv, lambda: gv.encode(model, X, "fp16"), "encode")
    n_srch = _sweep(gv, lambda: gv.search(model, ref_idx, Q, 10, 60), "search")
    assert n_enc > 0 and n_srch > 0
    idx = gv.encode(model, X, "fp16")
    got = gv.search(model, idx, Q, 10, 60)
    torch.cuda.synchronize()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    a, b = idx.export(), ref_idx.export()
    for key in ("tags", "offsets", "ids", "xlow", "scale"):
        assert np.array_equal(a[key], b[key]), key


def test_batched_search_survives_each_allocation_failure(gv, problem):
    X, QL, Q, model = problem
    idx = gv.encode(model, X, "bf16")
    ref = [gv.search(model, idx, Q[:m].contiguous(), 10, 40) for m in (90, 7)]
    gv.batch_release()
    Qs = [Q[:90].contiguous(), Q[:7].contiguous()]
    _sweep(gv, lambda: (gv.batch_release(), gv.search_batched([model, model], [idx, idx], Qs, 10, 40)), "batched")
    gv.batch_release()
    out = gv.search_batched([model, model], [idx, idx], Qs, 10, 40)
    torch.cuda.synchronize()
    for (i1, s1), (i2, s2) in zip(out, ref):
        assert torch.equal(i1, i2) and torch.equal(s1, s2)
    gv.batch_release()


def test_fit_survives_each_allocation_failure(gv, problem):
    X, QL, Q, model = problem
    sub = X[:8_000].contiguous()
    ref = gv.fit(sub, QL, 24, 4, seed=3)
    _sweep(gv, lambda: gv.fit(sub, QL, 24, 4, seed=3), "fit", limit=400)
    again = gv.fit(sub, QL, 24, 4, seed=3)
    for a, b in zip(ref.export(), again.export()):
        assert np.array_equal(a, b)
