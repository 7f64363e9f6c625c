"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
closed form, an invariant, a hand-derived worked instance (tests/golden), a
textbook routine, or brute force.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import formats
from oracle import gleanvec as G
from oracle.rng import SplitMix64, sample_without_replacement

RNG = np.random.default_rng(12345)


def _lowrank_data(rng, n, D, rank_scale=1.0, mean=None):
    """Anisotropic Gaussian rows with a decaying spectrum (full rank)."""
    lam = 1.0 / np.arange(1, D + 1)
    R, _ = np.linalg.qr(rng.standard_normal((D, D)))
    X = (rng.standard_normal((n, D)) * np.sqrt(lam)) @ R.T * rank_scale
    if mean is not None:
        X = X + mean
    return X


# ----------------------------------------------------------------------------- RNG

def test_splitmix64_published_vectors(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    for v in g["vectors"]:
        gen = SplitMix64(v["seed"])
        if "outputs_hex" in v:
            assert [gen.next() for _ in v["outputs_hex"]] == [int(h, 16) for h in v["outputs_hex"]]
        else:
            assert [gen.next() for _ in v["outputs"]] == v["outputs"]


def test_sample_without_replacement():
    gen = SplitMix64(7)
    s = sample_without_replacement(gen, 1000, 300)
    assert s.size == 300 and np.unique(s).size == 300 and s.min() >= 0 and s.max() < 1000
    assert np.all(np.diff(s) > 0)
    # every row equally likely: over many seeds the inclusion counts are flat
    counts = np.zeros(50)
    for seed in range(400):
        counts[sample_without_replacement(SplitMix64(seed), 50, 10)] += 1
    assert abs(counts.mean() - 80.0) < 1e-9 and counts.std() < 15
    assert np.array_equal(sample_without_replacement(SplitMix64(1), 10, 20), np.arange(10))


# ----------------------------------------------------------------------------- formats (T18)

@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8"])
def test_format_reference_values(golden_dir, fmt):
    g = json.load(open(os.path.join(golden_dir, "formats.json")))
    for code, val in g[fmt]:
        assert formats.decode(fmt, int(code, 16)) == val
        assert formats.round_to(fmt, val) == val
    if fmt == "fp8":
        for code in g["fp8_nan"]:
            assert np.isnan(formats.decode("fp8", int(code, 16)))


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8"])
def test_format_exhaustive_rne(fmt):
    """Every finite code is a fixed point; every midpoint between neighbours rounds
    to the neighbour with an even code; anything beyond max finite saturates."""
    nbits = 8 if fmt == "fp8" else 16
    codes = np.arange(1 << nbits)
    vals = formats.decode(fmt, codes)
    pos = codes[(vals > 0) & np.isfinite(vals) & ((codes >> (nbits - 1)) == 0)]
    pv = formats.decode(fmt, pos)
    order = np.argsort(pv)
    pos, pv = pos[order], pv[order]
    assert np.all(np.diff(pv) > 0)
    assert np.array_equal(formats.round_to(fmt, pv), pv)
    assert np.array_equal(formats.round_to(fmt, -pv), -pv)
    mid = 0.5 * (pv[:-1] + pv[1:])
    even = np.where(pos[:-1] % 2 == 0, pv[:-1], pv[1:])
    assert np.array_equal(formats.round_to(fmt, mid), even)
    # just off the midpoint goes to the nearer neighbour
    lo = mid - (pv[1:] - pv[:-1]) * 1e-3
    hi = mid + (pv[1:] - pv[:-1]) * 1e-3
    assert np.array_equal(formats.round_to(fmt, lo), pv[:-1])
    assert np.array_equal(formats.round_to(fmt, hi), pv[1:])
    # smallest subnormal: half of it ties to zero (even), above half goes up
    tiny = pv[0]
    assert formats.round_to(fmt, 0.5 * tiny) == 0.0
    assert formats.round_to(fmt, 0.75 * tiny) == tiny
    vmax = pv[-1]
    assert formats.SPECS[fmt][3] == vmax
    assert formats.round_to(fmt, vmax * 4) == vmax
    assert formats.round_to(fmt, -vmax * 4) == -vmax


def test_format_cross_check_numpy_fp16():
    x = RNG.standard_normal(200_000) * np.exp(RNG.uniform(-20, 12, 200_000))
    x = x[np.abs(x) < 65504]
    assert np.array_equal(formats.round_to("fp16", x), x.astype(np.float16).astype(np.float64))


def test_pow2_scale():
    for fmt, T in (("fp8", 448.0), ("fp16", 65504.0), ("bf16", 1.0)):
        amax = np.exp(RNG.uniform(-30, 30, 5000))
        amax = np.concatenate([amax, [T, T * 2, T / 2, T * 2 ** -10, T * 1.0000001]])
        s = formats.pow2_scale(fmt, amax)
        lg = np.log2(s)
        assert np.array_equal(lg, np.round(lg))
        r = amax / s
        assert np.all(r <= T) and np.all(r > T / 2)
    assert formats.pow2_scale("fp8", 0.0) == 1.0
    assert formats.pow2_scale("fp32", 123.0) == 1.0


# ----------------------------------------------------------------------------- top-k (T13)

def test_topk_brute_force_with_ties():
    rng = np.random.default_rng(3)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        k = int(rng.integers(1, n + 1))
        sc = rng.integers(-3, 4, n).astype(np.float64)   # many exact ties
        ids = rng.permutation(1000)[:n]
        got_ids, got_sc = G.topk(sc, ids, k)
        # brute force: repeatedly pick the best remaining by (score, then smaller id)
        rem = list(zip(sc.tolist(), ids.tolist()))
        want = []
        for _ in range(k):
            best = None
            for p in rem:
                if best is None or p[0] > best[0] or (p[0] == best[0] and p[1] < best[1]):
                    best = p
            want.append(best)
            rem.remove(best)
        assert got_ids.tolist() == [w[1] for w in want]
        assert got_sc.tolist() == [w[0] for w in want]
        # the definition of N (Section 2): every kept score >= every dropped score
        kept = set(got_ids.tolist())
        dropped = [s for s, i in zip(sc, ids) if i not in kept]
        if dropped:
            assert got_sc.min() >= max(dropped)


def test_exact_topk_streamed_vs_brute():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3000, 16)).astype(np.float32)
    Q = rng.standard_normal((5, 16)).astype(np.float32)
    ids, sc = G.exact_topk(X, Q, 10, chunk=256)
    for qi in range(5):
        full = X.astype(np.float64) @ Q[qi].astype(np.float64)
        want = sorted(range(3000), key=lambda i: (-full[i], i))[:10]
        assert ids[qi].tolist() == want


def test_recall_metric():
    truth = np.array([[1, 2, 3, 4, 5, 6, 7, 8, 9, 10]])
    assert G.recall(truth, truth) == 1.0
    assert G.recall(np.array([[1, 2, 3, 4, 5, 60, 70, 80, 90, 100]]), truth) == 0.5


# ----------------------------------------------------------------------------- k-means (T11, T12)

def test_kmeans_circle_golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "kmeans_circle.json")))
    ang = np.deg2rad(g["points_deg"])
    X = np.stack([np.cos(ang), np.sin(ang)], 1)
    a0 = np.deg2rad(g["init_deg"])
    mu0 = np.stack([np.cos(a0), np.sin(a0)], 1)
    mu, a, it = G.spherical_kmeans(X, mu0)
    ac = np.deg2rad(g["centres_deg"])
    assert np.allclose(mu, np.stack([np.cos(ac), np.sin(ac)], 1), atol=1e-15)
    assert a.tolist() == g["assignment"]


def test_tag_rule_equivalences():
    """T11: for unit landmarks, argmax <x, mu> = argmax <x/|x|, mu> = argmin |x - mu|
    (the VQ-VAE form of Section 4.2)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((2000, 24)) * rng.uniform(0.1, 10, (2000, 1))
    mu = G.normalise_rows(rng.standard_normal((7, 24)))
    a1 = G.assign(X, mu)
    a2 = G.assign(G.normalise_rows(X), mu)
    a3 = np.argmin(((X[:, None, :] - mu[None]) ** 2).sum(-1), axis=1)
    assert np.array_equal(a1, a2) and np.array_equal(a1, a3)
    # lowest index on exact ties
    mu2 = np.vstack([mu[:1], mu[:1], mu[1:]])
    assert np.all(G.assign(X, mu2) != 1)


def test_kmeans_monotone_and_fixed_point():
    """T12: the Appendix A objective never decreases over EM steps; at convergence the
    assignment is the arg-max and each centre is its members' normalised mean."""
    rng = np.random.default_rng(6)
    centres = G.normalise_rows(rng.standard_normal((6, 32)))
    X = centres[rng.integers(0, 6, 3000)] + 0.35 * rng.standard_normal((3000, 32)) / np.sqrt(32)
    Xt = G.normalise_rows(X)
    mu = G.kmeanspp(Xt, 6, SplitMix64(11))
    objs = [G.kmeans_objective(Xt, mu)]
    for _ in range(30):
        mu, a, it = G.spherical_kmeans(Xt, mu, max_iter=1)
        objs.append(G.kmeans_objective(Xt, mu))
    assert np.all(np.diff(objs) >= -1e-9)
    mu, a, it = G.spherical_kmeans(Xt, mu)
    assert np.array_equal(a, G.assign(Xt, mu))
    for c in range(6):
        s = Xt[a == c].sum(0)
        assert np.allclose(mu[c], s / np.linalg.norm(s), atol=1e-14)
    # recovery of the planted directions (well separated mixture)
    cos = np.max(np.abs(mu @ centres.T), axis=0)
    assert np.all(cos > 0.99)


def test_kmeanspp_draws_far_points():
    """k-means++ with C equal to the number of distinct points picks each exactly once
    (a point at chord distance 0 has zero probability)."""
    P = G.normalise_rows(np.eye(5) + 0.01)
    X = np.repeat(P, 40, axis=0)
    for seed in range(20):
        mu = G.kmeanspp(X, 5, SplitMix64(seed))
        assert np.unique(np.round(mu, 12), axis=0).shape[0] == 5


class _ScriptedDraws:
    """Stands in for the generator: returns the given integers and uniforms in order."""

    def __init__(self, ints, uniforms):
        self.ints = list(ints)
        self.uniforms = list(uniforms)

    def next(self):
        return self.ints.pop(0)

    def uniform(self):
        return self.uniforms.pop(0)


# Three unit points worked by hand: with the first centre at x0 = (1, 0), the
# squared chord distances 2 - 2 <x, x0> are 0, 2, 4 for x0, x1 = (0, 1),
# x2 = (-1, 0); their prefix sums are 0, 2, 6 of a total 6.  The D^2 law of
# k-means++ picks x1 with probability 2/6 and x2 with 4/6 (a law on the plain
# distance would give sqrt(2) / (sqrt(2) + 2) = 0.414 for x1).
_KPP_POINTS = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])


def test_kmeanspp_draw_follows_squared_distance_law():
    # exact picks for given uniforms: the first index whose prefix sum exceeds u * total
    for u, want in [(0.0, 1), (0.30, 1), (0.3333, 1), (0.334, 2), (0.9, 2)]:
        mu = G.kmeanspp(_KPP_POINTS, 2, _ScriptedDraws([0], [u]))
        assert np.array_equal(mu[1], _KPP_POINTS[want]), (u, want)
    # frequencies over SplitMix64 seeds whose first centre is x0
    picks = []
    seed = 0
    while len(picks) < 3000:
        gen = SplitMix64(seed)
        seed += 1
        probe = SplitMix64(gen.state)
        if probe.next() % 3 != 0:
            continue
        mu = G.kmeanspp(_KPP_POINTS, 2, gen)
        picks.append(int(np.argmax(_KPP_POINTS @ mu[1])))
    f1 = np.mean(np.array(picks) == 1)
    assert abs(f1 - 1.0 / 3.0) < 0.03, f1       # D^2 law: 1/3 (sd 0.009)
    assert abs(f1 - 0.414) > 0.05               # the plain-distance law is ruled out


def test_kmeanspp_tie_at_the_boundary_takes_the_next_point():
    """A uniform that lands exactly on a prefix sum: with x0 = (1, 0) first,
    x1 = (0, 1) and x2 = (0, -1) are both at squared chord distance 2; the prefix
    sums are 0, 2, 4 and u = 1/2 gives u * total = 2 exactly.  The draw takes the
    first index whose prefix sum strictly exceeds it, x2."""
    P = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, -1.0]])
    mu = G.kmeanspp(P, 2, _ScriptedDraws([0], [0.5]))
    assert np.array_equal(mu[1], P[2])
    mu = G.kmeanspp(P, 2, _ScriptedDraws([0], [0.4999999]))
    assert np.array_equal(mu[1], P[1])
    # the third centre of three: distances to the nearest of {x0, x2} are 0, 2, 0
    mu = G.kmeanspp(P, 3, _ScriptedDraws([0], [0.5, 0.99]))
    assert np.array_equal(mu[2], P[1])


# ----------------------------------------------------------------------------- sphering (T1-T10, T14-T16)

def _fitdata(seed, n=600, m=400, D=12):
    rng = np.random.default_rng(seed)
    X = _lowrank_data(rng, n, D)
    Q = _lowrank_data(rng, m, D)
    return Q, X


def test_golden_2d_query_aware(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "sphering_2d.json")))
    X = np.array(g["X"]); Q = np.array(g["Q"])
    KQ = G.second_moment(Q, mean=True)
    W, Wp, lamQ = G.sphering_W(KQ)
    assert np.allclose(W, g["W"], atol=1e-15)
    assert np.allclose(lamQ, g["eig_KQ"], atol=1e-15)
    P, lam = G.sphering_projection(W, G.second_moment(X, mean=False), g["d"])
    assert np.allclose(lam, g["eig_WKW"], atol=1e-14)
    A, B = P @ Wp, P @ W
    assert np.allclose(A, g["A"], atol=1e-15) and np.allclose(B, g["B"], atol=1e-15)
    assert np.allclose(A.T @ B, g["AtB"], atol=1e-15)
    L, _, _ = G.loss_pairwise(A[None], B[None], Q, [X], n_pairs=1.0)
    assert abs(L - g["loss_sum"]) < 1e-13
    L, _, _ = G.loss_pairwise(A[None], B[None], Q, [X])
    assert abs(L - g["loss_mean"]) < 1e-13
    U, _, _ = np.linalg.svd(X.T)
    pca = U[:, :1].T
    L, _, _ = G.loss_pairwise(pca[None], pca[None], Q, [X], n_pairs=1.0)
    assert abs(L - g["pca_loss_sum"]) < 1e-12


def test_T1_W_is_psd_root():
    Q, X = _fitdata(1)
    KQ = G.second_moment(Q, mean=True)
    W, Wp, _ = G.sphering_W(KQ)
    assert np.allclose(W, W.T, atol=1e-14)
    assert np.linalg.eigvalsh(W).min() > 0
    assert np.allclose(W @ W, KQ, atol=1e-13 * np.abs(KQ).max())
    assert np.allclose(W @ Wp, np.eye(12), atol=1e-11)
    # Eq. 6: Q Q^T = U S^2 U^T from the SVD of the stacked queries
    U, S, _ = np.linalg.svd(Q.T / np.sqrt(Q.shape[0]), full_matrices=False)
    assert np.allclose((U * S) @ U.T, W, atol=1e-12)


def test_T2_sphered_queries_are_white():
    Q, X = _fitdata(2)
    for d in (3, 7, 12):
        A, B = G.leanvec_sphering(Q, X, d)
        Z = Q @ A.T
        assert np.allclose(Z.T @ Z / Q.shape[0], np.eye(d), atol=1e-11)


def test_T3_reduced_database_moment_is_diagonal():
    Q, X = _fitdata(3)
    KQ = G.second_moment(Q, mean=True)
    W, Wp, _ = G.sphering_W(KQ)
    KX = G.second_moment(X, mean=False)
    P, lam = G.sphering_projection(W, KX, 5)
    B = P @ W
    Y = (X @ B.T).T @ (X @ B.T)
    assert np.allclose(Y, np.diag(lam[:5]), atol=1e-10 * lam[0])


def test_T4_full_dimension_is_exact():
    Q, X = _fitdata(4)
    A, B = G.leanvec_sphering(Q, X, 12)
    assert np.allclose(A.T @ B, np.eye(12), atol=1e-11)
    assert np.allclose((Q @ A.T) @ (X @ B.T).T, Q @ X.T, atol=1e-10)


def test_T5_T6_T7_loss_closed_form_gradient_zero_and_gram():
    """T5: the loss at the sphering solution is the Eckart-Young tail of W K_X W (with
    W from the summed K_Q); T6: its gradient vanishes (global minimiser of Problem 3
    over rank-d A^T B, by Eq. 5); T7: pairwise loss = Gram loss of Eq. 5."""
    rng = np.random.default_rng(7)
    D, d, C = 10, 4, 3
    Q = _lowrank_data(rng, 300, D)
    Xs = [_lowrank_data(rng, 200 + 50 * c, D, mean=rng.standard_normal(D)) for c in range(C)]
    KQs = G.second_moment(Q, mean=False)
    Ws, _, _ = G.sphering_W(KQs)
    A = np.empty((C, d, D)); B = np.empty((C, d, D))
    tail = 0.0
    for c in range(C):
        A[c], B[c] = G.leanvec_sphering(Q, Xs[c], d)
        lam = np.linalg.eigvalsh(Ws @ G.second_moment(Xs[c], False) @ Ws)
        tail += np.sort(lam)[::-1][d:].sum()
    L, dA, dB = G.loss_pairwise(A, B, Q, Xs, n_pairs=1.0)
    assert abs(L - tail) < 1e-9 * tail
    # gradient ~ 0 at the optimum, relative to the gradient at a perturbed point
    L2, dA2, dB2 = G.loss_pairwise(A + 0.01 * rng.standard_normal(A.shape), B, Q, Xs, n_pairs=1.0)
    assert np.linalg.norm(dA) < 1e-9 * np.linalg.norm(dA2)
    assert np.linalg.norm(dB) < 1e-9 * np.linalg.norm(dA2)
    # pairwise == Gram at a random point
    Ar = rng.standard_normal(A.shape); Br = rng.standard_normal(B.shape)
    KX = np.stack([G.second_moment(x, False) for x in Xs])
    N = Q.shape[0] * sum(x.shape[0] for x in Xs)
    Lp, dAp, dBp = G.loss_pairwise(Ar, Br, Q, Xs)
    Lg, dAg, dBg = G.loss_gram(Ar, Br, KQs, KX, N)
    assert abs(Lp - Lg) < 1e-12 * Lp
    assert np.allclose(dAp, dAg, rtol=1e-10, atol=1e-12 * np.abs(dAp).max())
    assert np.allclose(dBp, dBg, rtol=1e-10, atol=1e-12 * np.abs(dBp).max())


def test_T17_gradient_matches_central_differences():
    """The loss is quadratic in any single entry of A_c or B_c, so a central difference
    equals the derivative up to rounding for any step h."""
    rng = np.random.default_rng(8)
    D, d = 6, 3
    Q = rng.standard_normal((40, D))
    Xs = [rng.standard_normal((30, D)), rng.standard_normal((25, D))]
    A = rng.standard_normal((2, d, D)); B = rng.standard_normal((2, d, D))
    _, dA, dB = G.loss_pairwise(A, B, Q, Xs)
    h = 1e-3
    for (arr, grad) in ((A, dA), (B, dB)):
        for idx in [(0, 0, 0), (1, 2, 5), (0, 1, 3), (1, 0, 1)]:
            ap = arr.copy(); ap[idx] += h
            am = arr.copy(); am[idx] -= h
            args_p = (ap, B) if arr is A else (A, ap)
            args_m = (am, B) if arr is A else (A, am)
            fd = (G.loss_pairwise(*args_p, Q, Xs)[0] - G.loss_pairwise(*args_m, Q, Xs)[0]) / (2 * h)
            assert abs(fd - grad[idx]) < 1e-8 * max(1.0, abs(grad[idx]))


def test_T8_svd_route_equals_eigen_route():
    """Algorithm 2 as printed (SVD of Q, then SVD of W X) gives the same A^T B as the
    eigen route of Section 3.2."""
    Q, X = _fitdata(9)
    d = 5
    U, S, _ = np.linalg.svd(Q.T / np.sqrt(Q.shape[0]), full_matrices=False)
    W = (U * S) @ U.T
    Ux, _, _ = np.linalg.svd(W @ X.T, full_matrices=False)
    P = Ux[:, :d].T
    A1, B1 = P @ np.linalg.inv(W), P @ W
    A2, B2 = G.leanvec_sphering(Q, X, d)
    assert np.allclose(A1.T @ B1, A2.T @ B2, atol=1e-10)
    # and the same rows up to sign
    assert np.allclose(np.abs(A1), np.abs(A2), atol=1e-9)


def test_T10_isotropic_queries_reduce_to_pca():
    """With K_Q = alpha I, W = sqrt(alpha) I and A, B are (scaled) top-d left singular
    vectors of X: a truncated uncentered PCA."""
    rng = np.random.default_rng(10)
    D, d = 9, 4
    X = _lowrank_data(rng, 500, D)
    Q = np.sqrt(2.5 * D) * np.eye(D)            # K_Q (mean) = 2.5 I
    A, B = G.leanvec_sphering(Q, X, d)
    U, _, _ = np.linalg.svd(X.T, full_matrices=False)
    proj = U[:, :d] @ U[:, :d].T
    assert np.allclose(A.T @ B, proj, atol=1e-12)
    assert np.allclose(B / np.sqrt(2.5), A * np.sqrt(2.5), atol=1e-12)


def test_T14_scale_invariance():
    Q, X = _fitdata(11)
    A1, B1 = G.leanvec_sphering(Q, X, 5)
    A2, B2 = G.leanvec_sphering(Q * 7.0, X, 5)
    assert np.allclose(A1.T @ B1, A2.T @ B2, atol=1e-11)
    assert np.allclose(A2 * 7.0, A1, atol=1e-11)


def test_T15_pseudo_inverse_projects_on_query_span():
    rng = np.random.default_rng(12)
    D = 10
    Q = rng.standard_normal((6, D))        # rank 6 < D
    X = _lowrank_data(rng, 300, D)
    A, B = G.leanvec_sphering(Q, X, D)
    Pi = Q.T @ np.linalg.pinv(Q.T)         # projector onto span of the queries
    assert np.allclose(A.T @ B, Pi, atol=1e-10)
    q = rng.standard_normal(6) @ Q         # any query in the span is exact
    x = rng.standard_normal(D)
    assert abs((A @ q) @ (B @ x) - q @ x) < 1e-10 * np.linalg.norm(q) * np.linalg.norm(x)


def test_T16_nested_target_dimensions():
    """Section 3.1: the first d' rows of the d-solution are the d'-solution."""
    Q, X = _fitdata(13)
    A8, B8 = G.leanvec_sphering(Q, X, 8)
    A3, B3 = G.leanvec_sphering(Q, X, 3)
    assert np.allclose(A8[:3], A3, atol=1e-11) and np.allclose(B8[:3], B3, atol=1e-11)


def test_T9_one_cluster_is_leanvec_sphering():
    Q, X = _fitdata(14, n=900)
    m = G.fit(X, Q, 4, 1, seed=3)
    A, B = G.leanvec_sphering(Q, X, 4)
    assert np.allclose(m.A[0], A, atol=1e-12) and np.allclose(m.B[0], B, atol=1e-12)
    assert np.allclose(np.linalg.norm(m.mu, axis=1), 1.0)


def test_fit_gleanvec_properties():
    """Algorithm 5 end to end: unit landmarks, per-cluster sphering, and a loss no larger
    than the single-projection (C = 1) solution on the learn data."""
    rng = np.random.default_rng(15)
    D, d, C = 16, 4, 3
    means = G.normalise_rows(rng.standard_normal((C, D))) * 3
    X = np.concatenate([_lowrank_data(rng, 400, D, mean=means[c]) for c in range(C)])
    Q = _lowrank_data(rng, 500, D)
    m = G.fit(X, Q, d, C, seed=5)
    assert np.allclose(np.linalg.norm(m.mu, axis=1), 1.0)
    assert m.counts.sum() == X.shape[0] and not m.fallback.any()
    tags = G.assign(X, m.mu)
    Xs = [X[tags == c] for c in range(C)]
    Lg, _, _ = G.loss_pairwise(m.A, m.B, Q, Xs)
    m1 = G.fit(X, Q, d, 1, seed=5)
    L1, _, _ = G.loss_pairwise(m1.A, m1.B, Q, [X])
    assert Lg <= L1 * (1 + 1e-12)
    # each cluster's projection is the sphering solution of its own member set (T2 holds)
    for c in range(C):
        Z = Q @ m.A[c].T
        assert np.allclose(Z.T @ Z / Q.shape[0], np.eye(d), atol=1e-10)


def test_fit_fallback_for_tiny_cluster():
    rng = np.random.default_rng(16)
    D, d = 8, 5
    X = np.concatenate([_lowrank_data(rng, 300, D, mean=3 * np.eye(D)[0]),
                        3 * np.eye(D)[1] + 0.01 * rng.standard_normal((3, D))])
    Q = _lowrank_data(rng, 200, D)
    mu0 = np.stack([np.eye(D)[0], np.eye(D)[1]])
    m = G.fit(X, Q, d, 2, seed=1, mu0=mu0)
    assert m.counts.tolist() == [300, 3] and m.fallback.tolist() == [False, True]
    A, B = G.leanvec_sphering(Q, X, d)
    assert np.allclose(m.A[1], A, atol=1e-12)


# ----------------------------------------------------------------------------- encode and search

def _small_problem(fmt, seed=20, n=3000, D=24, d=8, C=4, m=7):
    rng = np.random.default_rng(seed)
    means = G.normalise_rows(rng.standard_normal((C, D))) * 2
    X = np.concatenate([_lowrank_data(rng, n // C, D, mean=means[c]) for c in range(C)]).astype(np.float32)
    Q = _lowrank_data(rng, m, D).astype(np.float32)
    QL = _lowrank_data(rng, 400, D).astype(np.float32)
    model = G.fit(X, QL, d, C, seed=2)
    return model, X, Q


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
def test_encode_definition(fmt):
    model, X, Q = _small_problem(fmt)
    idx = G.encode(model.mu, model.B, X, fmt)
    n = X.shape[0]
    # grouping: a permutation, clusters contiguous, stable (increasing ids inside)
    assert np.array_equal(np.sort(idx.ids), np.arange(n))
    for c in range(model.C):
        seg = idx.ids[idx.offsets[c]:idx.offsets[c + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(idx.tags[seg] == c)
    # brute-force per row: x_low = B_c x for c = arg-max tag, one FP32 rounding
    for p in RNG.integers(0, n, 50):
        i = idx.ids[p]
        c = int(np.argmax([float(np.dot(X[i].astype(np.float64), model.mu[cc])) for cc in range(model.C)]))
        assert idx.tags[i] == c
        exact = np.array([sum(float(model.B[c, j, t]) * float(X[i, t]) for t in range(X.shape[1]))
                          for j in range(model.d)])
        assert np.allclose(idx.v[p], exact, rtol=2 ** -23, atol=0)
        s = idx.scale[c]
        assert np.all(np.abs(idx.xq[p] * s - idx.v[p]) <= np.abs(idx.v[p]) * (2 ** -3 if fmt == "fp8" else 2 ** -7) + s * 2 ** -6)
    # the per-cluster scale from its definition: a power of two putting the cluster's
    # largest |v| into (T/2, T] (T = 448, 65504, 1; FP32 unscaled)
    T = {"fp32": None, "fp16": 65504.0, "bf16": 1.0, "fp8": 448.0}[fmt]
    for c in range(model.C):
        a, b = idx.offsets[c], idx.offsets[c + 1]
        s = idx.scale[c]
        if T is None or a == b:
            assert s == 1.0
            continue
        amax = np.abs(idx.v[a:b]).max()
        mant, _ = math.frexp(s)
        assert mant == 0.5, s                       # a power of two
        assert T / 2 < amax / s <= T, (c, amax, s)
        assert np.abs(idx.xq[a:b]).max() <= T        # no saturation was needed
    # every stored value is the nearest value of the format to v / s (ties to even),
    # checked against the format's grid written out from its definition
    M, emin = {"fp32": (23, -126), "fp16": (10, -14), "bf16": (7, -126), "fp8": (3, -6)}[fmt]
    for c in range(model.C):
        a, b = idx.offsets[c], idx.offsets[c + 1]
        y = (idx.v[a:b] / idx.scale[c]).ravel()
        got = idx.xq[a:b].ravel()
        e = np.array([max(math.frexp(abs(v))[1] - 1, emin) if v != 0 else emin for v in y])
        q = np.ldexp(1.0, e - M)                  # spacing of the grid around each value
        lo = np.floor(y / q) * q
        hi = lo + q
        dlo, dhi = y - lo, hi - y
        want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi,
                        np.where(np.mod(np.round(lo / q), 2) == 0, lo, hi)))
        assert np.array_equal(got, want), fmt
    if fmt == "fp16":   # a second opinion: numpy's own binary16 conversion
        for c in range(model.C):
            a, b = idx.offsets[c], idx.offsets[c + 1]
            y = idx.v[a:b] / idx.scale[c]
            assert np.array_equal(idx.xq[a:b], y.astype(np.float16).astype(np.float64))


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
def test_search_stages_against_brute_force(fmt):
    model, X, Q = _small_problem(fmt, seed=21)
    idx = G.encode(model.mu, model.B, X, fmt)
    k, kappa = 5, 40
    out = G.search(idx, model.A, Q, k, kappa)
    n = X.shape[0]
    pos_of = np.empty(n, np.int64); pos_of[idx.ids] = np.arange(n)
    for qi in range(Q.shape[0]):
        # reduced score of every vector by plain loops over Eq. 11 with the eager views
        s = np.empty(n)
        for i in range(n):
            c = idx.tags[i]
            p = pos_of[i]
            s[i] = idx.scale[c] * out["t"][qi, c] * sum(out["qh"][qi, c, j] * idx.xq[p, j] for j in range(model.d))
        want = sorted(range(n), key=lambda i: (-s[i], i))[:kappa]
        assert out["cand_ids"][qi].tolist() == want
        exact = {i: float(np.dot(X[i].astype(np.float64), Q[qi].astype(np.float64))) for i in want}
        final = sorted(want, key=lambda i: (-exact[i], i))[:k]
        assert out["ids"][qi].tolist() == final
    # the FP32 view approximates the exact A_c q
    qc_exact = np.einsum("cjD,mD->mcj", model.A, Q.astype(np.float64))
    assert np.allclose(out["qc"], qc_exact, rtol=2 ** -23, atol=0)


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
def test_query_view_definition(fmt):
    """The query view: t a power of two putting max_j |q_c,j| into (T/2, T] of the
    view format, q^ the nearest value of that format to q_c / t.  FP8 storage meets
    FP16 views, checked against numpy's own binary16 rounding; FP32 is unscaled."""
    model, X, Q = _small_problem(fmt, seed=23)
    qc, t, qh = G.project_queries(model.A, Q, fmt)
    exact = np.einsum("cjD,mD->mcj", model.A, Q.astype(np.float64))
    assert np.array_equal(qc, exact.astype(np.float32).astype(np.float64))
    if fmt == "fp32":
        assert np.all(t == 1.0) and np.array_equal(qh, qc)
        return
    T = {"fp16": 65504.0, "bf16": 1.0, "fp8": 65504.0}[fmt]
    amax = np.abs(qc).max(axis=2)
    assert np.all((T / 2 < amax / t) & (amax / t <= T))
    assert np.all(np.frexp(t)[0] == 0.5)
    y = qc / t[:, :, None]
    if fmt in ("fp16", "fp8"):
        assert np.array_equal(qh, y.astype(np.float16).astype(np.float64))
    else:  # bf16: nearest of the 8-bit-significand grid, ties to even
        e = np.maximum(np.frexp(np.abs(y))[1] - 1, -126)
        q = np.ldexp(1.0, e - 7)
        lo = np.floor(y / q) * q
        want = np.where(y - lo < lo + q - y, lo, np.where(y - lo > lo + q - y, lo + q,
                        np.where(np.mod(np.round(lo / q), 2) == 0, lo, lo + q)))
        assert np.array_equal(qh, want)


def test_search_full_dimension_recovers_exact_topk():
    """T4 through the whole search: with d = D, FP32 storage and kappa = k the reduced
    scores equal the exact inner products up to FP32 rounding, so the result is the
    exact top-k (checked on queries whose k-th gap is wide)."""
    rng = np.random.default_rng(22)
    D = 16
    X = _lowrank_data(rng, 2000, D).astype(np.float32)
    Q = _lowrank_data(rng, 20, D).astype(np.float32)
    model = G.fit(X, _lowrank_data(rng, 300, D), D, 1, seed=4)
    idx = G.encode(model.mu, model.B, X, "fp32")
    out = G.search(idx, model.A, Q, 10, 10)
    gt, gs = G.exact_topk(X, Q, 11)
    for qi in range(Q.shape[0]):
        if gs[qi, 9] - gs[qi, 10] > 1e-4 * abs(gs[qi, 0]):
            assert set(out["ids"][qi].tolist()) == set(gt[qi, :10].tolist())
        assert np.allclose(out["cand_scores"][qi], np.sort(out["out_scores"][qi])[::-1], rtol=1e-5, atol=1e-5)


# ----------------------------------------------------------------------------- flexible d (Section 3.3)

def test_flex_leading_coordinates_equal_refit_at_smaller_d():
    """Searching the leading 3 of 8 stored coordinates is the search of the model fitted
    at d = 3 (Section 3.3 with the nesting of Section 3.1): same views, same reduced
    scores up to FP32 rounding of the stored rows, same final top-k."""
    model8, X, Q = _small_problem("fp32", seed=30)
    rng = np.random.default_rng(30)
    QL = _lowrank_data(rng, 400, X.shape[1]).astype(np.float32)
    model8 = G.fit(X, QL, 8, 4, seed=2)
    model3 = G.fit(X, QL, 3, 4, seed=2)
    assert not model8.fallback.any()
    assert np.allclose(model8.A[:, :3], model3.A, atol=1e-12) and np.allclose(model8.B[:, :3], model3.B, atol=1e-12)
    i8 = G.encode(model8.mu, model8.B, X, "fp32")
    i3 = G.encode(model3.mu, model3.B, X, "fp32")
    assert np.array_equal(i8.ids, i3.ids) and np.allclose(i8.xq[:, :3], i3.xq, rtol=2 ** -22, atol=0)
    k, kappa = 5, 40
    f = G.search_flex(i8, model8.A, Q, k, kappa, 3, "full")
    r = G.search(i3, model3.A, Q, k, kappa)
    assert np.allclose(f["qh"], r["qh"], rtol=2 ** -22, atol=0)
    assert np.allclose(f["cand_scores"], r["cand_scores"], rtol=1e-6, atol=1e-9)
    assert np.array_equal(f["ids"], r["ids"])


def test_flex_stored_rerank_at_full_dimension_is_exact():
    """Section 3.3: with d_s = D the stored vectors give undistorted similarities,
    <A' q, x'> = <q, x> (A'^T B' = I when K_Q has full rank), cluster by cluster."""
    rng = np.random.default_rng(31)
    D = 12
    means = G.normalise_rows(rng.standard_normal((2, D))) * 2
    X = np.concatenate([_lowrank_data(rng, 600, D, mean=means[c]) for c in range(2)]).astype(np.float32)
    Q = _lowrank_data(rng, 6, D).astype(np.float32)
    model = G.fit(X, _lowrank_data(rng, 300, D), D, 2, seed=5)
    idx = G.encode(model.mu, model.B, X, "fp32")
    out = G.search_flex(idx, model.A, Q, 5, 30, 4, "stored")
    for qi in range(Q.shape[0]):
        ci = out["cand_ids"][qi]
        got = G.rerank_stored(idx, out["qc"], qi, ci)
        exact = X[ci].astype(np.float64) @ Q[qi].astype(np.float64)
        assert np.allclose(got, exact, rtol=1e-5, atol=1e-5 * np.abs(exact).max())
        assert np.array_equal(out["ids"][qi], G.topk(got, ci, 5)[0])


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "fp8"])
def test_flex_stages_against_brute_force(fmt):
    """Leading-coordinate scores and the stored rerank by plain loops over Eq. 11 and
    the Section 3.3 identity."""
    model, X, Q = _small_problem(fmt, seed=32)
    idx = G.encode(model.mu, model.B, X, fmt)
    ds, k, kappa = 5, 4, 30
    out = G.search_flex(idx, model.A, Q, k, kappa, ds, "stored")
    n = X.shape[0]
    pos_of = np.empty(n, np.int64); pos_of[idx.ids] = np.arange(n)
    qc_exact = np.einsum("cjD,mD->mcj", model.A, Q.astype(np.float64))
    assert np.allclose(out["qc"], qc_exact, rtol=2 ** -23, atol=0) and out["qc"].shape[2] == model.d
    for qi in range(Q.shape[0]):
        amax = np.abs(out["qc"][qi, :, :ds]).max(axis=1)
        # the scale of the leading d_search values (FP8 storage: FP16 views, T = 65504)
        assert np.array_equal(out["t"][qi], formats.pow2_scale("fp16" if fmt == "fp8" else fmt, amax))
        s = np.empty(n)
        for i in range(n):
            c = idx.tags[i]
            p = pos_of[i]
            s[i] = idx.scale[c] * out["t"][qi, c] * sum(out["qh"][qi, c, j] * idx.xq[p, j] for j in range(ds))
        want = sorted(range(n), key=lambda i: (-s[i], i))[:kappa]
        assert out["cand_ids"][qi].tolist() == want
        st = {i: sum(out["qc"][qi, idx.tags[i], j] * idx.xq[pos_of[i], j] * idx.scale[idx.tags[i]]
                     for j in range(model.d)) for i in want}
        assert out["ids"][qi].tolist() == sorted(want, key=lambda i: (-st[i], i))[:k]


# ----------------------------------------------------------------------------- Euclidean adaptation (Appendix)

def test_euclidean_augmentation_identity_and_nearest_neighbours():
    """<q^, x^> = <q, x> - ||x||^2 / 2 (up to the one FP32 rounding of the appended
    value), so the arg-max of the augmented inner product is the Euclidean nearest
    neighbour: checked against scipy's distances by brute force."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(40)
    X = (rng.standard_normal((500, 7)) * rng.uniform(0.2, 3.0, (500, 1))).astype(np.float32)
    Q = rng.standard_normal((30, 7)).astype(np.float32)
    Xa = G.augment_database(X)
    Qa = G.augment_queries(Q)
    assert Xa.dtype == np.float32 and Xa.shape == (500, 8) and np.array_equal(Xa[:, :7], X)
    assert np.array_equal(Qa[:, :7], Q) and np.all(Qa[:, 7] == 1.0)
    ip = Qa.astype(np.float64) @ Xa.astype(np.float64).T
    want = Q.astype(np.float64) @ X.astype(np.float64).T - 0.5 * np.sum(X.astype(np.float64) ** 2, axis=1)
    assert np.allclose(ip, want, rtol=0, atol=2 ** -24 * np.abs(want).max() * 2)
    dist = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    for qi in range(30):
        order = np.argsort(dist[qi], kind="stable")
        if dist[qi, order[1]] - dist[qi, order[0]] > 1e-4:
            assert int(np.argmax(ip[qi])) == int(order[0])
        # the whole ranking agrees where the gaps are wide
        a = np.argsort(-ip[qi], kind="stable")[:10]
        gaps = np.diff(dist[qi, order[:11]])
        if np.all(gaps > 1e-4):
            assert a.tolist() == order[:10].tolist()


def test_euclidean_search_end_to_end():
    """Fit, encode and search on augmented vectors (FP32 storage, d = D + 1): the
    result is the Euclidean top-k where the k-th gap is wide."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(41)
    D = 10
    X = (_lowrank_data(rng, 1500, D) * rng.uniform(0.3, 2.0, (1500, 1))).astype(np.float32)
    Q = _lowrank_data(rng, 15, D).astype(np.float32)
    QL = _lowrank_data(rng, 300, D).astype(np.float32)
    Xa, Qa, QLa = G.augment_database(X), G.augment_queries(Q), G.augment_queries(QL)
    model = G.fit(Xa, QLa, D + 1, 2, seed=6)
    idx = G.encode(model.mu, model.B, Xa, "fp32")
    out = G.search(idx, model.A, Qa, 5, 40)
    dist = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    checked = 0
    for qi in range(15):
        order = np.argsort(dist[qi], kind="stable")
        if dist[qi, order[5]] - dist[qi, order[4]] > 1e-3 * dist[qi, order[4]]:
            assert set(out["ids"][qi].tolist()) == set(order[:5].tolist())
            checked += 1
    assert checked >= 8


# ----------------------------------------------------------------------------- streaming updates (Section 3)

def test_streaming_moment_updates_are_exact():
    """Adding the inserted vectors' outer products and subtracting the removed ones
    gives the statistics of the final set (integer data: every sum is exact)."""
    rng = np.random.default_rng(60)
    X0 = rng.integers(-8, 9, (300, 6)).astype(np.float64)
    ins = rng.integers(-8, 9, (50, 6)).astype(np.float64)
    tags0 = rng.integers(0, 3, 300); tags_ins = rng.integers(0, 3, 50)
    rm = rng.choice(300, 40, replace=False)
    K0 = np.stack([X0[tags0 == c].T @ X0[tags0 == c] for c in range(3)])
    K = G.update_moments(K0, ins, tags_ins, +1)
    K = G.update_moments(K, X0[rm], tags0[rm], -1)
    keep = np.setdiff1d(np.arange(300), rm)
    Xf = np.concatenate([X0[keep], ins]); tf = np.concatenate([tags0[keep], tags_ins])
    want = np.stack([Xf[tf == c].T @ Xf[tf == c] for c in range(3)])
    assert np.array_equal(K, want)


def test_fit_from_stats_equals_fit_with_kept_landmarks():
    """The projections recomputed from the statistics of a set are those of fitting the
    set with the landmarks held fixed (no Lloyd step)."""
    model, X, Q = _small_problem("fp32", seed=61)
    rng = np.random.default_rng(61)
    QL = _lowrank_data(rng, 400, X.shape[1]).astype(np.float32)
    ref = G.fit(X, QL, 5, 4, seed=2, mu0=model.mu, max_iter=0)
    tags = G.assign(X.astype(np.float64), model.mu)
    KX = np.stack([G.second_moment(X[tags == c], mean=False) for c in range(4)])
    KQs = G.second_moment(QL, mean=False)
    got = G.fit_from_stats(model.mu, KQs, QL.shape[0], KX, np.bincount(tags, minlength=4), 5)
    assert np.allclose(got.A, ref.A, atol=1e-10) and np.allclose(got.B, ref.B, atol=1e-10)
    assert np.array_equal(got.fallback, ref.fallback)


# ----------------------------------------------------------------------------- streaming re-projection (Section 3)

def _stream_models(seed=41, D=12, C=3):
    rng = np.random.default_rng(seed)
    means = G.normalise_rows(rng.standard_normal((C, D))) * 2
    X0 = np.concatenate([_lowrank_data(rng, 400, D, mean=means[c]) for c in range(C)]).astype(np.float32)
    Xn = np.concatenate([_lowrank_data(rng, 60, D, mean=means[c]) for c in range(C)]).astype(np.float32)
    QL = _lowrank_data(rng, 500, D).astype(np.float32)
    m0 = G.fit(X0, QL, D, C, seed=3)
    keep = np.ones(X0.shape[0], bool)
    keep[rng.choice(X0.shape[0], 90, replace=False)] = False
    t0 = G.assign(X0.astype(np.float64), m0.mu)
    tn = G.assign(Xn.astype(np.float64), m0.mu)
    K = G.update_moments(m0.KX, Xn, tn, +1)
    K = G.update_moments(K, X0[~keep], t0[~keep], -1)
    QL2 = _lowrank_data(rng, 300, D).astype(np.float32)
    KQ = G.second_moment(np.concatenate([QL, QL2]), mean=False)
    counts = np.bincount(np.concatenate([t0[keep], tn]), minlength=C)
    m1 = G.fit_from_stats(m0.mu, KQ, QL.shape[0] + QL2.shape[0], K, counts, D)
    return X0, Xn, keep, m0, m1


def test_reproject_equals_fresh_encode_at_full_rank():
    """With every coordinate stored (d = D) and K_Q of full rank, P'W'(PW)^-1 applied to
    the stored P W x is P'W'x: the re-projected index equals a fresh encode of the
    current set with the refitted model, up to the FP32 rounding of the stored values
    carried through the transform; removed ids are gone, inserted ones take the next
    ids and the arg-max tag of the kept landmarks."""
    X0, Xn, keep, m0, m1 = _stream_models()
    n0, D = X0.shape
    idx0 = G.encode(m0.mu, m0.B, X0, "fp32")
    re = G.reproject_index(idx0, m0.mu, m0.A, m1.B, "fp32", X_new=Xn, keep=keep)
    X_all = np.concatenate([X0, Xn])
    present = np.concatenate([keep, np.ones(Xn.shape[0], bool)])
    # fresh encode of the current set, mapped back to the id space
    cur_ids = np.nonzero(present)[0]
    fresh = G.encode(m1.mu, m1.B, X_all[cur_ids], "fp32")
    assert np.all(re.tags[~present] == 255)
    assert np.array_equal(re.tags[present], fresh.tags)
    assert np.array_equal(re.ids, cur_ids[fresh.ids])
    assert np.array_equal(re.offsets, fresh.offsets)
    err = np.abs(re.v - fresh.v).max(axis=1) / np.linalg.norm(fresh.v, axis=1)
    assert err.max() < 1e-5, err.max()
    # kept vectors keep their cluster
    assert np.array_equal(re.tags[:n0][keep], idx0.tags[keep])


def test_reproject_with_the_same_model_keeps_the_stored_values():
    """With no refit, B_c A_c^T = P W W+ P^T = I (d = D, full rank): every stored value
    comes back, up to the FP64 rounding of the identity."""
    X0, Xn, keep, m0, m1 = _stream_models(seed=43)
    for fmt in ("fp32", "fp16"):
        idx0 = G.encode(m0.mu, m0.B, X0, fmt)
        re = G.reproject_index(idx0, m0.mu, m0.A, m0.B, fmt)
        assert np.array_equal(re.ids, idx0.ids) and np.array_equal(re.offsets, idx0.offsets)
        y = idx0.xq * idx0.scale[np.repeat(np.arange(idx0.scale.shape[0]), np.diff(idx0.offsets))][:, None]
        same = re.v == y
        assert same.mean() > 0.999
        assert np.all(np.abs(re.v - y) <= np.spacing(np.abs(y).astype(np.float32)).astype(np.float64) + 1e-30)
