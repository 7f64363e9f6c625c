"""Loss and gradient of the per-cluster projections on the GPU (the
differentiable-refinement row): statistics, tags, loss and gradient against the
FP64 oracle's pairwise and Gram forms, central differences, the closed-form
minimum, and the autograd wrapper used to refine a sphering fit."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import gleanvec as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U32 = 2.0 ** -24
U64 = 2.0 ** -53


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


def _mixture(cfg, D, J, n, m):
    geom = synth.make_geometry(cfg, D, J, "mixture")
    X = synth.database(geom, n)
    Q = synth.queries(geom, m, synth.S_QTEST)
    QL = synth.queries(geom, m, synth.S_QLEARN)
    return X, Q, QL


def _oracle_tags(X, mu):
    return np.argmax(np.asarray(X, np.float64) @ mu.T, axis=1)


def _oracle_stats(Q, X, tags, C):
    KQ = G.second_moment(Q, mean=False)
    KX = np.stack([G.second_moment(X[tags == c], mean=False) for c in range(C)])
    return KQ, KX


def test_moments_match_oracle(gv):
    """K[c] = sum over rows tagged c of v v^T, FP64: exact products, so the only error
    is the summation order (n * 2^-53 relative to sum |v_i v_j|)."""
    _say("[loss] moments")
    rng = np.random.default_rng(11)
    n, D, C = 6000, 64, 5
    V = rng.standard_normal((n, D)).astype(np.float32)
    tags = rng.integers(0, C, n).astype(np.uint8)
    tags[:7] = 3  # a cluster present; cluster sizes ragged
    K = gv.moments(dev(V), dev(tags), C).cpu().numpy()
    Va = np.abs(V.astype(np.float64))
    for c in range(C):
        ref = G.second_moment(V[tags == c], mean=False)
        scale = Va[tags == c].T @ Va[tags == c]
        assert np.all(np.abs(K[c] - ref) <= n * U64 * scale + 1e-300)
    K1 = gv.moments(dev(V)).cpu().numpy()[0]
    assert np.all(np.abs(K1 - G.second_moment(V, False)) <= n * U64 * (Va.T @ Va))
    # empty input
    assert np.all(gv.moments(dev(V[:0]), dev(tags[:0]), C).cpu().numpy() == 0.0)


def test_tags_match_oracle(gv):
    """Cluster tags from the oracle's centroids: bit-exact where the top-two gap
    exceeds the FP64 dot-product error bound."""
    _say("[loss] tags")
    X, Q, QL = _mixture(301, 96, 6, 20_000, 500)
    om = G.fit(X, QL, 24, 6, seed=3)
    model = gv.model_import(om.mu, om.A, om.B)
    t_gpu = gv.tags(model, dev(X)).cpu().numpy()
    dots = np.asarray(X, np.float64) @ om.mu.T
    t_ora = np.argmax(dots, axis=1)
    srt = np.sort(dots, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    tol = 2 * X.shape[1] * U64 * (np.abs(X.astype(np.float64)) @ np.abs(om.mu).T).max(axis=1)
    clear = gap > tol
    assert clear.mean() > 0.99
    assert np.array_equal(t_gpu[clear], t_ora[clear])


def _random_problem(seed, C, d, D, m, nc):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((m, D)) @ np.diag(1.0 / np.sqrt(np.arange(1, D + 1)))
    Xs = [rng.standard_normal((nc + 37 * c, D)) @ np.diag(1.0 / np.arange(1, D + 1) ** 0.4) + 0.3 * rng.standard_normal(D)
          for c in range(C)]
    A = np.empty((C, d, D)); B = np.empty((C, d, D))
    for c in range(C):
        A[c], B[c] = G.leanvec_sphering(Q, Xs[c], d)
    A = (A + 0.05 * rng.standard_normal(A.shape) * np.abs(A).mean()).astype(np.float32)
    B = (B + 0.05 * rng.standard_normal(B.shape) * np.abs(B).mean()).astype(np.float32)
    return Q, Xs, A, B


def _loss_scale(KQ, KX, N):
    """Size of the terms the Gram form cancels: sum_c <|K_Q|, |K_c|> / N."""
    return sum(np.sum(np.abs(KQ) * np.abs(k)) for k in KX) / N


@pytest.mark.parametrize("C,d,D", [(3, 12, 48), (2, 40, 130)])
def test_loss_grad_matches_oracle(gv, C, d, D):
    """GPU loss/gradient vs the oracle's Gram form (M_c = A^T B - I) and the pairwise
    definition, on the same FP32 parameters and FP64 statistics."""
    _say(f"[loss] grad C{C} d{d} D{D}")
    Q, Xs, A, B = _random_problem(21 + D, C, d, D, 600, 300)
    KQ = G.second_moment(Q, False)
    KX = np.stack([G.second_moment(x, False) for x in Xs])
    N = Q.shape[0] * sum(x.shape[0] for x in Xs)
    loss, dA, dB = gv.loss_grad(dev(A), dev(B), dev(KQ), dev(KX), N)
    loss = float(loss.cpu()); dA = dA.cpu().numpy(); dB = dB.cpu().numpy()
    Lg, dAg, dBg = G.loss_gram(A.astype(np.float64), B.astype(np.float64), KQ, KX, N)
    Lp, dAp, dBp = G.loss_pairwise(A.astype(np.float64), B.astype(np.float64), Q, Xs, N)
    assert abs(Lg - Lp) <= 1e-10 * Lp
    scale = _loss_scale(KQ, KX, N)
    assert abs(loss - Lg) <= 64 * D * U64 * scale, (loss, Lg, scale)
    for g, ref in ((dA, dAg), (dB, dBg)):
        err = np.abs(g - ref)
        assert np.all(err <= U32 * np.abs(ref) + 1e-9 * np.abs(ref).max()), err.max()
    # loss only
    l2, a2, b2 = gv.loss_grad(dev(A), dev(B), dev(KQ), dev(KX), N, grads=False)
    assert a2 is None and b2 is None and float(l2.cpu()) == loss


def test_loss_gradient_central_differences(gv):
    """The loss is quadratic in each entry of A_c or B_c, so a central difference of the
    GPU loss equals the GPU gradient up to rounding; checked on entries of the block
    rows 0-63 x columns 0-255 of one cluster."""
    _say("[loss] central differences")
    C, d, D = 2, 64, 256
    Q, Xs, A, B = _random_problem(5, C, d, D, 800, 600)
    KQ = dev(G.second_moment(Q, False))
    KX = dev(np.stack([G.second_moment(x, False) for x in Xs]))
    N = Q.shape[0] * sum(x.shape[0] for x in Xs)
    scale = _loss_scale(G.second_moment(Q, False), [G.second_moment(x, False) for x in Xs], N)
    Ad, Bd = dev(A), dev(B)
    _, dA, dB = gv.loss_grad(Ad, Bd, KQ, KX, N)
    dA = dA.cpu().numpy(); dB = dB.cpu().numpy()
    rng = np.random.default_rng(9)
    h = 1e-3
    for which, P, g in (("A", A, dA), ("B", B, dB)):
        for _ in range(12):
            idx = (1, int(rng.integers(0, 64)), int(rng.integers(0, 256)))
            ap = P.copy(); ap[idx] = np.float32(P[idx] + h)
            am = P.copy(); am[idx] = np.float32(P[idx] - h)
            args_p = (dev(ap), Bd) if which == "A" else (Ad, dev(ap))
            args_m = (dev(am), Bd) if which == "A" else (Ad, dev(am))
            lp = float(gv.loss_grad(*args_p, KQ, KX, N, grads=False)[0].cpu())
            lm = float(gv.loss_grad(*args_m, KQ, KX, N, grads=False)[0].cpu())
            fd = (lp - lm) / (float(ap[idx]) - float(am[idx]))
            tol = 2 * 64 * D * U64 * scale / (2 * h) + U32 * abs(g[idx])
            assert abs(fd - g[idx]) <= tol, (which, idx, fd, g[idx], tol)


def test_autograd_refinement_reaches_toward_closed_form(gv):
    """Refinement of a sphering fit (learned on a separate query set) on training
    pairs through the autograd wrapper: the training loss decreases and stays above
    its closed-form minimum (the sphering solution of the training statistics)."""
    _say("[loss] refinement")
    D, C, d = 64, 4, 12
    X, QT, QL = _mixture(302, D, C, 16_000, 3_000)
    om = G.fit(X, QL, d, C, seed=4)
    Xd, Qd = dev(X), dev(QT)
    t_ora = _oracle_tags(X, om.mu)  # both sides use the oracle's tags
    KQ = gv.moments(Qd)[0]
    KX = gv.moments(Xd, dev(t_ora.astype(np.uint8)), C)
    N = QT.shape[0] * X.shape[0]
    # closed form on the training statistics (oracle): Eckart-Young tails of W K_c W
    KQo, KXo = _oracle_stats(QT, X, t_ora, C)
    Ws, _, _ = G.sphering_W(KQo)
    Lstar = sum(np.sort(np.linalg.eigvalsh(Ws @ KXo[c] @ Ws))[::-1][d:].sum() for c in range(C)) / N
    A = torch.tensor(om.A.astype(np.float32), device="cuda", requires_grad=True)
    B = torch.tensor(om.B.astype(np.float32), device="cuda", requires_grad=True)
    L0 = float(gv.gleanvec_loss(A, B, KQ, KX, N))
    # the wrapper's gradient is the library's
    loss = gv.gleanvec_loss(A, B, KQ, KX, N)
    loss.backward()
    _, dA, dB = gv.loss_grad(A.detach(), B.detach(), KQ, KX, N)
    assert torch.equal(A.grad, dA) and torch.equal(B.grad, dB)
    A.grad = None; B.grad = None
    opt = torch.optim.LBFGS([A, B], lr=1.0, max_iter=40, history_size=20, line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        loss = gv.gleanvec_loss(A, B, KQ, KX, N)
        loss.backward()
        return loss

    opt.step(closure)
    L1 = float(gv.gleanvec_loss(A, B, KQ, KX, N))
    _say(f"[loss] refinement: L* {Lstar:.6g}  start {L0:.6g}  end {L1:.6g}")
    assert L0 > Lstar
    assert L1 < L0
    assert L1 >= Lstar * (1 - 1e-9)
    assert (L1 - Lstar) < 0.5 * (L0 - Lstar)


def test_loss_grad_full_shape(gv):
    """The refinement shape (C = 32, D = 768, d = 128): GPU loss and gradient against
    the oracle's Gram form on the same statistics; reports the time per call."""
    _say("[loss] full shape")
    C, d, D = 32, 128, 768
    rng = np.random.default_rng(13)
    geom = synth.make_geometry(305, D, C, "mixture")
    X = synth.database(geom, 64_000)
    QT = synth.queries(geom, 4_000, synth.S_QTRAIN)
    tags = rng.integers(0, C, X.shape[0])  # any partition: the identity holds per cluster
    KQ, KX = _oracle_stats(QT, X, tags, C)
    A = (rng.standard_normal((C, d, D)) / np.sqrt(D)).astype(np.float32)
    B = (rng.standard_normal((C, d, D)) / np.sqrt(D)).astype(np.float32)
    N = QT.shape[0] * X.shape[0]
    Ad, Bd, KQd, KXd = dev(A), dev(B), dev(KQ), dev(KX)
    loss, dA, dB = gv.loss_grad(Ad, Bd, KQd, KXd, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        gv.loss_grad(Ad, Bd, KQd, KXd, N)
    torch.cuda.synchronize()
    _say(f"[loss] C32 d128 D768 loss+grad: {(time.perf_counter() - t0) / 5 * 1e3:.3f} ms per call")
    Lg, dAg, dBg = G.loss_gram(A.astype(np.float64), B.astype(np.float64), KQ, KX, N)
    scale = _loss_scale(KQ, KX, N)
    assert abs(float(loss.cpu()) - Lg) <= 64 * D * U64 * scale
    for g, ref in ((dA.cpu().numpy(), dAg), (dB.cpu().numpy(), dBg)):
        assert np.all(np.abs(g - ref) <= U32 * np.abs(ref) + 1e-9 * np.abs(ref).max())


def test_refinement_at_stated_scale(gv):
    """The refinement workload at its full scale: C = 32, D = 768, d = 128, statistics
    from 100,000 OOD training queries and 1,000,000 database vectors (drawn on the
    device), starting from a sphering fit.  The GPU loss and gradient agree with the
    oracle's Gram form on the same statistics; central differences (h = 1e-3) of the
    GPU loss agree with the GPU gradient on 96 entries of the 64 x 256 slice of one
    cluster, for A and for B; the autograd wrapper's gradient is the library's; and
    a short L-BFGS refinement lowers the training loss while staying above its
    closed-form minimum.  Reports the time per loss + gradient call."""
    _say("[loss] stated scale")
    C, d, D = 32, 128, 768
    n, mq = 1_000_000, 100_000
    geom = synth.make_geometry(306, D, C, "mixture")
    X = synth.draw_torch(geom, n, synth.S_DB, "cuda")
    QT = synth.draw_torch(geom, mq, synth.S_QTRAIN, "cuda", queries_=True)
    QL = synth.draw_torch(geom, 20_000, synth.S_QLEARN, "cuda", queries_=True)
    rows = torch.from_numpy(synth.learn_rows(n, 100_000, 306)).cuda()
    model = gv.fit(X[rows].contiguous(), QL, d, C, seed=5)
    t = gv.tags(model, X)
    KQ = gv.moments(QT)[0]
    KX = gv.moments(X, t, C)
    N = float(mq) * float(n)
    _, Af, Bf = model.export()
    A0 = torch.tensor(np.asarray(Af, np.float32), device="cuda")
    B0 = torch.tensor(np.asarray(Bf, np.float32), device="cuda")
    loss, dA, dB = gv.loss_grad(A0, B0, KQ, KX, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        gv.loss_grad(A0, B0, KQ, KX, N)
    torch.cuda.synchronize()
    _say(f"[loss] stated scale: {(time.perf_counter() - t0) / 5 * 1e3:.3f} ms per loss + gradient call")
    KQh, KXh = KQ.cpu().numpy(), KX.cpu().numpy()
    A, B = A0.cpu().numpy(), B0.cpu().numpy()
    Lg, dAg, dBg = G.loss_gram(A.astype(np.float64), B.astype(np.float64), KQh, KXh, N)
    scale = _loss_scale(KQh, KXh, N)
    assert abs(float(loss.cpu()) - Lg) <= 64 * D * U64 * scale
    dA = dA.cpu().numpy(); dB = dB.cpu().numpy()
    for g, ref in ((dA, dAg), (dB, dBg)):
        assert np.all(np.abs(g - ref) <= U32 * np.abs(ref) + 1e-9 * np.abs(ref).max())
    # central differences on the 64 x 256 slice (rows 0-63, columns 0-255) of cluster 7
    rng = np.random.default_rng(21)
    h = 1e-3
    for which, P, g in (("A", A, dA), ("B", B, dB)):
        for _ in range(96):
            idx = (7, int(rng.integers(0, 64)), int(rng.integers(0, 256)))
            ap = P.copy(); ap[idx] = np.float32(P[idx] + h)
            am = P.copy(); am[idx] = np.float32(P[idx] - h)
            args_p = (dev(ap), B0) if which == "A" else (A0, dev(ap))
            args_m = (dev(am), B0) if which == "A" else (A0, dev(am))
            lp = float(gv.loss_grad(*args_p, KQ, KX, N, grads=False)[0].cpu())
            lm = float(gv.loss_grad(*args_m, KQ, KX, N, grads=False)[0].cpu())
            fd = (lp - lm) / (float(ap[idx]) - float(am[idx]))
            tol = 2 * 64 * D * U64 * scale / (2 * h) + U32 * abs(g[idx])
            assert abs(fd - g[idx]) <= tol, (which, idx, fd, g[idx], tol)
    # the autograd wrapper, then a short refinement against the closed-form minimum
    Ws, _, _ = G.sphering_W(KQh)
    Lstar = sum(np.sort(np.linalg.eigvalsh(Ws @ KXh[c] @ Ws))[::-1][d:].sum() for c in range(C)) / N
    Ap = A0.clone().requires_grad_(True)
    Bp = B0.clone().requires_grad_(True)
    L0 = gv.gleanvec_loss(Ap, Bp, KQ, KX, N)
    L0.backward()
    assert torch.equal(Ap.grad, torch.from_numpy(dA).cuda()) and torch.equal(Bp.grad, torch.from_numpy(dB).cuda())
    Ap.grad = None; Bp.grad = None
    # the objective is the loss relative to its start (its gradient entries at this
    # scale lie below L-BFGS's default stopping tolerance)
    L0v = float(L0)
    opt = torch.optim.LBFGS([Ap, Bp], lr=1.0, max_iter=10, history_size=10, line_search_fn="strong_wolfe",
                            tolerance_grad=0.0, tolerance_change=0.0)

    def closure():
        opt.zero_grad()
        loss = gv.gleanvec_loss(Ap, Bp, KQ, KX, N) / L0v
        loss.backward()
        return loss

    opt.step(closure)
    L1 = float(gv.gleanvec_loss(Ap, Bp, KQ, KX, N))
    _say(f"[loss] stated scale: L* {Lstar:.6g}  start {float(L0):.6g}  after 10 L-BFGS steps {L1:.6g}")
    assert float(L0) > Lstar and L1 < float(L0) and L1 >= Lstar * (1 - 1e-9)
