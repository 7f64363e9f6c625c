"""FP64 oracle of GleanVec / LeanVec-Sphering: fit, encode and search.

Test infrastructure only.  Written from the paper (GleanVec, arXiv
2410.22347); each function names the passage it follows.  Inputs are FP32
arrays (the paper's datasets are FP32, Table 1) and are upcast to float64;
all arithmetic is float64 unless a step states a cast.  Nothing here is
blocked, fused or reordered beyond the definitions, so it can be checked
against the paper by eye.

Readings of points the paper leaves open (also listed in the design notes):

* second moments are uncentered; K_Q is the mean of q q^T (Section 3.2 writes
  a sum -- the projections A^T B are invariant to the scale), K_{X_c} the sum;
* the pseudo-inverse of W (Section 3) drops eigenvalues below D * 2^-52 * lambda_max;
* eigenvectors are sorted by decreasing eigenvalue; each row of P_c is
  sign-fixed so that its largest-magnitude entry (lowest index on ties) is
  positive;
* arg-max ties go to the lowest cluster index; top-k ties to the lowest id;
* spherical k-means: at most 50 Lloyd steps, stop when no assignment changes,
  an empty cluster keeps its centre; k-means++ uses the squared chord
  distance 2 - 2 <x~, mu> on the sphere;
* a cluster with fewer than d learn vectors uses the projection fitted on
  the pooled learn set (the C = 1 solution) -- a rank-deficient K_{X_c}
  would leave P_c undetermined;
* storage formats and scales (not in the paper): per-cluster power-of-two
  scale s_c for the database and per-(query, cluster) scale t for the query
  view, both mapping the block's amax into (T/2, T], then round-to-nearest-even
  (see ``formats``); FP8 storage meets FP16 query views (``VIEW_FORMAT``).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import formats
from .rng import SplitMix64, sample_without_replacement

KMEANS_SAMPLE = 100_000
KMEANS_MAX_ITER = 50


# ============================================================================ top-k
def topk(scores: np.ndarray, ids: np.ndarray, k: int):
    """The k best (score, id) pairs, ordered by score desc then id asc.

    The paper's top-k (Section 2, definition of the set N) allows any set on
    exact ties; the canonical order picks the lowest ids.
    """
    order = np.lexsort((ids, -scores))[:k]
    return ids[order], scores[order]


# ============================================================================ k-means
def normalise_rows(X: np.ndarray) -> np.ndarray:
    """x~ = x / |x|_2 (Algorithm 5, first step; Appendix A); zero rows stay zero."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt(np.sum(X * X, axis=1))
    out = np.zeros_like(X)
    nz = nrm > 0
    out[nz] = X[nz] / nrm[nz, None]
    return out


def assign(Xt: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """c_i = argmax_c <x_i, mu_c> (Eq. 9 / Appendix A E-step), lowest c on ties."""
    return np.argmax(np.asarray(Xt, np.float64) @ mu.T, axis=1)


def kmeanspp(Xt: np.ndarray, C: int, gen: SplitMix64) -> np.ndarray:
    """k-means++ seeding on the sphere (Appendix A): the first centre uniform,
    each next one drawn with probability proportional to the squared chord
    distance to the nearest chosen centre."""
    n = Xt.shape[0]
    first = gen.next() % n
    mu = [Xt[first].copy()]
    best = Xt @ mu[0]
    for _ in range(1, C):
        d2 = np.maximum(0.0, 2.0 - 2.0 * best)
        cum = np.cumsum(d2)              # sequential float64 prefix sum
        total = cum[-1]
        u = gen.uniform()
        if total > 0:
            i = int(np.argmax(cum > u * total))   # first index strictly above
        else:
            i = int(u * n)
        mu.append(Xt[i].copy())
        best = np.maximum(best, Xt @ mu[-1])
    return np.array(mu)


def spherical_kmeans(Xt: np.ndarray, mu0: np.ndarray, max_iter: int = KMEANS_MAX_ITER):
    """Lloyd iterations of spherical k-means (Appendix A): assign by arg-max inner
    product, then mu_c = normalised sum of its members.  Returns (mu, assignment,
    number of centre updates)."""
    mu = mu0.copy()
    a = assign(Xt, mu)
    it = 0
    for it in range(1, max_iter + 1):
        for c in range(mu.shape[0]):
            members = Xt[a == c]
            if members.shape[0] == 0:
                continue
            s = members.sum(axis=0)
            nrm = np.sqrt(np.sum(s * s))
            if nrm > 0:
                mu[c] = s / nrm
        new = assign(Xt, mu)
        if np.array_equal(new, a):
            break
        a = new
    return mu, a, it


def kmeans_objective(Xt: np.ndarray, mu: np.ndarray) -> float:
    """sum_i max_c <x~_i, mu_c> (Appendix A objective, to be maximised)."""
    return float(np.max(Xt @ mu.T, axis=1).sum())


# ============================================================================ sphering
def second_moment(V: np.ndarray, mean: bool) -> np.ndarray:
    """Uncentered second moment sum_v v v^T (Section 3.2 statistics); /count if mean."""
    V = np.asarray(V, np.float64)
    K = V.T @ V
    if mean and V.shape[0] > 0:
        K = K / V.shape[0]
    return K


def eigh_desc(K: np.ndarray):
    lam, U = np.linalg.eigh(K)
    return lam[::-1].copy(), U[:, ::-1].copy()


def sphering_W(KQ: np.ndarray, rcond: float | None = None):
    """W = U S U^T with U S^2 U^T = K_Q (Eq. 6), and its pseudo-inverse (Section 3)."""
    D = KQ.shape[0]
    lam, U = eigh_desc(KQ)
    S = np.sqrt(np.maximum(lam, 0.0))
    if rcond is None:
        rcond = D * 2.0 ** -52
    keep = lam > rcond * lam[0] if lam[0] > 0 else np.zeros(D, bool)
    Sp = np.zeros(D)
    Sp[keep] = 1.0 / S[keep]
    W = (U * S) @ U.T
    Wp = (U * Sp) @ U.T
    return W, Wp, lam


def canonical_signs(P: np.ndarray) -> np.ndarray:
    """Flip each row so its largest-magnitude entry (lowest index on ties) is positive."""
    P = P.copy()
    for r in range(P.shape[0]):
        j = int(np.argmax(np.abs(P[r])))
        if P[r, j] < 0:
            P[r] = -P[r]
    return P


def sphering_projection(W: np.ndarray, KX: np.ndarray, d: int):
    """P = top-d eigenvectors (as rows) of W K_X W (Section 3.2, replacing the SVD of
    W X in Algorithm 2).  Returns (P, eigenvalues in decreasing order)."""
    Y = W @ KX @ W
    Y = 0.5 * (Y + Y.T)
    lam, V = eigh_desc(Y)
    P = canonical_signs(V[:, :d].T)
    return P, lam


def leanvec_sphering(Q: np.ndarray, X: np.ndarray, d: int):
    """Algorithm 2 (LeanVec-Sphering) through the eigen route of Section 3.2.
    Returns A, B (d x D)."""
    KQ = second_moment(Q, mean=True)
    KX = second_moment(X, mean=False)
    W, Wp, _ = sphering_W(KQ)
    P, _ = sphering_projection(W, KX, d)
    return P @ Wp, P @ W


@dataclasses.dataclass
class Model:
    mu: np.ndarray        # C x D, unit rows
    A: np.ndarray         # C x d x D
    B: np.ndarray         # C x d x D
    W: np.ndarray
    Wp: np.ndarray
    lam_Q: np.ndarray     # eigenvalues of K_Q, decreasing
    lam_c: np.ndarray     # C x D eigenvalues of W K_{X_c} W, decreasing
    counts: np.ndarray    # learn vectors per cluster
    fallback: np.ndarray  # bool per cluster: used the pooled projection
    KQ: np.ndarray
    KX: np.ndarray        # C x D x D (sums)
    kmeans_iters: int = 0

    @property
    def C(self):
        return self.mu.shape[0]

    @property
    def d(self):
        return self.A.shape[1]

    @property
    def D(self):
        return self.A.shape[2]


def fit(X_learn: np.ndarray, Q_learn: np.ndarray, d: int, C: int, seed: int,
        mu0: np.ndarray | None = None, kmeans_sample: int = KMEANS_SAMPLE,
        max_iter: int = KMEANS_MAX_ITER) -> Model:
    """GleanVec learning (Algorithm 5): spherical k-means landmarks on the
    normalised learn set, then LeanVec-Sphering (Algorithm 2, eigen route of
    Section 3.2) for each cluster with one shared W from the learn queries."""
    X = np.asarray(X_learn, np.float64)
    Qm = np.asarray(Q_learn, np.float64)
    D = X.shape[1]
    gen = SplitMix64(seed)
    # --- landmarks (Appendix A): k-means on a uniform sample of the normalised set
    sample = sample_without_replacement(gen, X.shape[0], kmeans_sample)
    Xt = normalise_rows(X[sample])
    if mu0 is None:
        mu0 = kmeanspp(Xt, C, gen)
    mu, _, iters = spherical_kmeans(Xt, np.asarray(mu0, np.float64), max_iter)
    # --- partition of the learn set (Algorithm 5; Eq. 9 on unnormalised vectors)
    tags = assign(X, mu)
    # --- statistics (Section 3.2)
    KQ = second_moment(Qm, mean=True)
    KX = np.stack([second_moment(X[tags == c], mean=False) for c in range(C)])
    counts = np.bincount(tags, minlength=C)
    return projections_from_stats(mu, KQ, KX, counts, d, iters)


def projections_from_stats(mu: np.ndarray, KQ: np.ndarray, KX: np.ndarray, counts: np.ndarray, d: int,
                           iters: int = 0) -> Model:
    """Per-cluster LeanVec-Sphering from the second-moment statistics (Section 3.2,
    Algorithm 2 through eigendecompositions): KQ the mean of q q^T, KX the per-cluster
    sums of x x^T; a cluster with fewer than d vectors takes the pooled projection."""
    C, D = mu.shape
    counts = np.asarray(counts, np.int64)
    W, Wp, lam_Q = sphering_W(KQ)
    A = np.empty((C, d, D))
    B = np.empty((C, d, D))
    lam_c = np.empty((C, D))
    fallback = counts < d
    if fallback.any():
        P_pool, lam_pool = sphering_projection(W, KX.sum(axis=0), d)
    for c in range(C):
        if fallback[c]:
            P, lam = P_pool, lam_pool
        else:
            P, lam = sphering_projection(W, KX[c], d)
        A[c] = P @ Wp
        B[c] = P @ W
        lam_c[c] = lam
    return Model(mu, A, B, W, Wp, lam_Q, lam_c, counts, fallback, KQ, KX, iters)


# ============================================================================ streaming
# Section 3 (streaming vector search): the statistics are sums, so inserting or
# removing x adds or subtracts x x^T; the projections are recomputed from them
# (the SVDs of Algorithm 2 replaced by eigendecompositions) with the landmarks kept.

def update_moments(K: np.ndarray, V: np.ndarray, tags: np.ndarray | None, sign: int) -> np.ndarray:
    """K[c] + sign * sum_{v with tag c} v v^T, float64 (tags None: one cluster)."""
    K = np.array(K, np.float64, copy=True)
    V = np.asarray(V, np.float64)
    tags = np.zeros(V.shape[0], np.int64) if tags is None else np.asarray(tags)
    for c in range(K.shape[0]):
        Vc = V[tags == c]
        K[c] += sign * (Vc.T @ Vc)
    return K


def fit_from_stats(mu: np.ndarray, KQ_sum: np.ndarray, m_q: float, KX: np.ndarray, counts: np.ndarray,
                   d: int) -> Model:
    """The model of kept landmarks and statistics: K_Q = KQ_sum / m_q."""
    return projections_from_stats(np.asarray(mu, np.float64), np.asarray(KQ_sum, np.float64) / m_q,
                                  np.asarray(KX, np.float64), counts, d)


def reproject_index(index: "Index", mu: np.ndarray, A_old: np.ndarray, B_new: np.ndarray, fmt: str,
                    X_new: np.ndarray | None = None, keep: np.ndarray | None = None) -> "Index":
    """Streaming re-projection of stored vectors (Section 3, streaming vector
    search).  The index stores y = P_c W x with every coordinate (d = D, the
    flexible storage of Section 3.3).  After a refit, the kept vectors become
    P'_c W' (P_c W)^-1 y, where (P_c W)^-1 = W^-1 P_c^T is A_c^T = (P_c W+)^T
    (P_c orthogonal, K_Q of full rank); inserted vectors x become P'_c W' x =
    B'_c x; removed ones are dropped.  The landmarks mu are unchanged, so kept
    vectors keep their tag.  Stored values y are s_c x^ (exact); each new value
    is the float64 product rounded once to FP32, then scaled per cluster and
    rounded to fmt as in encode.  The result keeps no full-dimension vectors;
    removed ids get tag 255."""
    C = mu.shape[0]
    n_old = index.tags.shape[0]
    X_new = np.zeros((0, A_old.shape[2]), np.float32) if X_new is None else np.asarray(X_new, np.float32)
    tags = np.concatenate([np.asarray(index.tags, np.int64), assign(np.asarray(X_new, np.float64), mu)])
    if keep is not None:
        tags[:n_old][~np.asarray(keep, bool)] = 255
    present = np.nonzero(tags < C)[0]
    ids = present[np.argsort(tags[present], kind="stable")].astype(np.int64)   # by (tag, id)
    counts = np.bincount(tags[present], minlength=C)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pos_old = np.empty(n_old, np.int64)
    pos_old[index.ids] = np.arange(index.ids.shape[0])
    d = B_new.shape[1]
    v = np.empty((ids.shape[0], d))
    xq = np.empty((ids.shape[0], d))
    scale = np.ones(C)
    for c in range(C):
        rows = ids[offsets[c]:offsets[c + 1]]
        T = np.asarray(B_new[c], np.float64) @ np.asarray(A_old[c], np.float64).T
        vc = np.empty((rows.shape[0], d))
        for r, i in enumerate(rows):
            if i < n_old:
                y = index.xq[pos_old[i]] * index.scale[c]          # the stored vector, exactly
                vc[r] = T @ y
            else:
                vc[r] = np.asarray(B_new[c], np.float64) @ X_new[i - n_old].astype(np.float64)
        vc = formats.round_to("fp32", vc)
        v[offsets[c]:offsets[c + 1]] = vc
        amax = np.max(np.abs(vc)) if vc.size else 0.0
        s = float(formats.pow2_scale(fmt, amax))
        scale[c] = s
        xq[offsets[c]:offsets[c + 1]] = formats.round_to(fmt, vc / s)
    out_tags = np.where(tags < C, tags, 255).astype(np.int64)
    return Index(fmt, out_tags, offsets, ids, v, xq, scale, None)


# ============================================================================ encode
@dataclasses.dataclass
class Index:
    fmt: str
    tags: np.ndarray      # n, cluster of each original row
    offsets: np.ndarray   # C + 1, grouped segment boundaries
    ids: np.ndarray       # n, original row id of each grouped position
    v: np.ndarray         # n x d, fl32(B_c x) in grouped order (float64 holding FP32 values)
    xq: np.ndarray        # n x d, stored values x^ (float64 holding fmt values), grouped order
    scale: np.ndarray     # C, per-cluster power-of-two scale s_c
    X: np.ndarray | None  # n x D original vectors (FP32), original order; None when not kept


def encode(model_mu: np.ndarray, B: np.ndarray, X: np.ndarray, fmt: str) -> Index:
    """Tags (Eq. 9) and reduced vectors x^low = B_{c_i} x_i (Eq. 10, read with g_c),
    grouped by cluster, then quantised with a per-cluster scale."""
    X64 = np.asarray(X, np.float64)
    C = model_mu.shape[0]
    tags = assign(X64, model_mu)
    ids = np.argsort(tags, kind="stable").astype(np.int64)   # by (tag, id)
    counts = np.bincount(tags, minlength=C)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    B64 = np.asarray(B, np.float64)
    d = B.shape[1]
    v = np.empty((X.shape[0], d))
    xq = np.empty((X.shape[0], d))
    scale = np.ones(C)
    for c in range(C):
        rows = ids[offsets[c]:offsets[c + 1]]
        vc = formats.round_to("fp32", X64[rows] @ B64[c].T)
        v[offsets[c]:offsets[c + 1]] = vc
        amax = np.max(np.abs(vc)) if vc.size else 0.0
        s = float(formats.pow2_scale(fmt, amax))
        scale[c] = s
        xq[offsets[c]:offsets[c + 1]] = formats.round_to(fmt, vc / s)
    return Index(fmt, tags, offsets, ids, v, xq, scale, np.asarray(X, np.float32))


# ============================================================================ search
# Format of the query view q^ that meets the stored vectors in the reduced inner
# product (not in the paper): the storage format itself, except FP8 storage,
# whose scores are formed with FP16 query views -- FP16 x E4M3 products are
# exact, so FP8 storage halves the bytes read without rounding the query to
# three fraction bits.
VIEW_FORMAT = {"fp32": "fp32", "fp16": "fp16", "bf16": "bf16", "fp8": "fp16"}


def project_queries(A: np.ndarray, Q: np.ndarray, fmt: str):
    """Eager preprocessing (Algorithm 4, preprocess): q_c = A_c q for every c in
    float64, rounded once to FP32; then the per-(query, cluster) power-of-two
    scale t and the view q^ = rnd(q_c / t) in VIEW_FORMAT[fmt].
    Returns (q_c [m, C, d], t [m, C], q^ [m, C, d])."""
    A64 = np.asarray(A, np.float64)
    Q64 = np.asarray(Q, np.float64)
    C, d, D = A64.shape
    qc = formats.round_to("fp32", (Q64 @ A64.reshape(C * d, D).T).reshape(-1, C, d))
    amax = np.max(np.abs(qc), axis=2)
    vf = VIEW_FORMAT[fmt]
    t = formats.pow2_scale(vf, amax)
    qh = formats.round_to(vf, qc / t[:, :, None])
    return qc, t, qh


def reduced_scores(index: Index, t: np.ndarray, qh: np.ndarray) -> np.ndarray:
    """Eq. 11 with the eager views (Algorithm 4, inner-product): for x_i in cluster c,
    s_i = s_c * t_{q,c} * <q^_c, x^_i>, in float64.  Returns m x n in grouped order."""
    m = qh.shape[0]
    n = index.xq.shape[0]
    out = np.empty((m, n))
    for c in range(index.offsets.shape[0] - 1):
        a, b = index.offsets[c], index.offsets[c + 1]
        if a == b:
            continue
        out[:, a:b] = (qh[:, c, :] @ index.xq[a:b].T) * (index.scale[c] * t[:, c])[:, None]
    return out


def search(index: Index, A: np.ndarray, Q: np.ndarray, k: int, kappa: int):
    """Multi-step search (Algorithm 1) with a brute-force main step: preprocess (eager
    views), retrieve the kappa best reduced scores, rerank them with exact full-D inner
    products and keep the top k.  Returns a dict with every stage's output."""
    qc, t, qh = project_queries(A, Q, index.fmt)
    S = reduced_scores(index, t, qh)
    m = Q.shape[0]
    cand_ids = np.empty((m, kappa), np.int64)
    cand_sc = np.empty((m, kappa))
    out_ids = np.empty((m, k), np.int64)
    out_sc = np.empty((m, k))
    Q64 = np.asarray(Q, np.float64)
    for qi in range(m):
        ci, cs = topk(S[qi], index.ids, kappa)
        cand_ids[qi], cand_sc[qi] = ci, cs
        exact = np.asarray(index.X[ci], np.float64) @ Q64[qi]
        oi, os_ = topk(exact, ci, k)
        out_ids[qi], out_sc[qi] = oi, os_
    return dict(qc=qc, t=t, qh=qh, scores=S, cand_ids=cand_ids, cand_scores=cand_sc,
                ids=out_ids, out_scores=out_sc)


# ============================================================================ Euclidean distance
# Appendix (adapting other similarities): nearest neighbours under the Euclidean
# distance become maximum inner products after appending one coordinate,
# x^ = [x, -||x||^2 / 2] and q^ = [q, 1], since <q^, x^> = <q, x> - ||x||^2 / 2
# differs from -||q - x||^2 / 2 by a term constant in x.

def augment_database(X: np.ndarray) -> np.ndarray:
    """[x, -||x||^2 / 2] per row; the norm in float64 from the FP32 values, the
    appended value rounded once to FP32.  Returns FP32, n x (D + 1)."""
    X32 = np.asarray(X, np.float32)
    sq = np.sum(X32.astype(np.float64) ** 2, axis=1)
    return np.concatenate([X32, formats.round_to("fp32", -0.5 * sq)[:, None].astype(np.float32)], axis=1)


def augment_queries(Q: np.ndarray) -> np.ndarray:
    """[q, 1] per row, FP32, m x (D + 1)."""
    Q32 = np.asarray(Q, np.float32)
    return np.concatenate([Q32, np.ones((Q32.shape[0], 1), np.float32)], axis=1)


# ============================================================================ flexible d
# Section 3.3: the stored vectors keep d_s >= d coordinates ordered by decreasing
# eigenvalue of W K_X W (the rows of P come sorted that way), so a search may use
# any leading d of them, fixed at search time; and the stored vectors themselves
# can serve the rerank, <q, x> ~ <A q, x'> with x' the stored coordinates (exact
# when d_s = D and K_Q has full rank, since then A^T B = I).

def project_queries_flex(A: np.ndarray, Q: np.ndarray, fmt: str, d_search: int):
    """Eager views on the leading d_search coordinates: q_c = fl32(A_c q) over all
    d_s stored rows (the rerank from stored vectors uses them all); the scale t and
    the view q^ (in VIEW_FORMAT[fmt]) come from the first d_search values only.
    Returns (q_c [m, C, d_s], t [m, C], q^ [m, C, d_search])."""
    A64 = np.asarray(A, np.float64)
    Q64 = np.asarray(Q, np.float64)
    C, d, D = A64.shape
    assert 1 <= d_search <= d
    qc = formats.round_to("fp32", (Q64 @ A64.reshape(C * d, D).T).reshape(-1, C, d))
    lead = qc[:, :, :d_search]
    vf = VIEW_FORMAT[fmt]
    t = formats.pow2_scale(vf, np.max(np.abs(lead), axis=2))
    qh = formats.round_to(vf, lead / t[:, :, None])
    return qc, t, qh


def reduced_scores_flex(index: Index, t: np.ndarray, qh: np.ndarray, d_search: int) -> np.ndarray:
    """Eq. 11 on the leading d_search stored coordinates: for x_i in cluster c,
    s_i = s_c * t_{q,c} * sum_{j < d_search} q^_{c,j} x^_{i,j}, float64, grouped order."""
    m = qh.shape[0]
    n = index.xq.shape[0]
    out = np.empty((m, n))
    for c in range(index.offsets.shape[0] - 1):
        a, b = index.offsets[c], index.offsets[c + 1]
        if a == b:
            continue
        out[:, a:b] = (qh[:, c, :d_search] @ index.xq[a:b, :d_search].T) * (index.scale[c] * t[:, c])[:, None]
    return out


def rerank_stored(index: Index, qc: np.ndarray, q: int, cand_ids: np.ndarray):
    """Rerank of one query's candidates from the stored vectors (Section 3.3):
    <A_c q, x'_i> = sum_j q_{c,j} * (s_c x^_{i,j}) over every stored coordinate,
    float64, c the candidate's cluster.  Returns the scores of cand_ids."""
    pos_of = np.full(index.tags.shape[0], -1, np.int64)   # id -> stored row (ids may have gaps)
    pos_of[index.ids] = np.arange(index.ids.shape[0])
    out = np.empty(cand_ids.shape[0])
    for r, i in enumerate(cand_ids):
        c = index.tags[i]
        out[r] = float(np.dot(qc[q, c], index.xq[pos_of[i]] * index.scale[c]))
    return out


def search_flex(index: Index, A: np.ndarray, Q: np.ndarray, k: int, kappa: int, d_search: int,
                rerank: str = "full"):
    """Algorithm 1 with the reduced dimension chosen at search time (Section 3.3):
    the main step scores the leading d_search coordinates; the rerank uses the full
    vectors (rerank = "full") or the stored ones (rerank = "stored")."""
    qc, t, qh = project_queries_flex(A, Q, index.fmt, d_search)
    S = reduced_scores_flex(index, t, qh, d_search)
    m = Q.shape[0]
    cand_ids = np.empty((m, kappa), np.int64)
    cand_sc = np.empty((m, kappa))
    out_ids = np.empty((m, k), np.int64)
    out_sc = np.empty((m, k))
    Q64 = np.asarray(Q, np.float64)
    for qi in range(m):
        ci, cs = topk(S[qi], index.ids, kappa)
        cand_ids[qi], cand_sc[qi] = ci, cs
        if rerank == "stored":
            exact = rerank_stored(index, qc, qi, ci)
        else:
            exact = np.asarray(index.X[ci], np.float64) @ Q64[qi]
        oi, os_ = topk(exact, ci, k)
        out_ids[qi], out_sc[qi] = oi, os_
    return dict(qc=qc, t=t, qh=qh, scores=S, cand_ids=cand_ids, cand_scores=cand_sc,
                ids=out_ids, out_scores=out_sc)


def exact_topk(X: np.ndarray, Q: np.ndarray, k: int, chunk: int = 1 << 18):
    """Ground truth: the k largest <q, x_i> over all i (Section 2), float64, streamed
    over row chunks with a running merge."""
    Q64 = np.asarray(Q, np.float64)
    m = Q64.shape[0]
    best_ids = np.zeros((m, 0), np.int64)
    best_sc = np.zeros((m, 0))
    for s in range(0, X.shape[0], chunk):
        blk = np.asarray(X[s:s + chunk], np.float64)
        sc = Q64 @ blk.T
        ids = np.arange(s, s + blk.shape[0], dtype=np.int64)
        new_ids = np.empty((m, min(k, best_ids.shape[1] + ids.size)), np.int64)
        new_sc = np.empty(new_ids.shape)
        for qi in range(m):
            allsc = np.concatenate([best_sc[qi], sc[qi]])
            allid = np.concatenate([best_ids[qi], ids])
            new_ids[qi], new_sc[qi] = topk(allsc, allid, k)
        best_ids, best_sc = new_ids, new_sc
    return best_ids, best_sc


def recall(found: np.ndarray, truth: np.ndarray, K: int = 10) -> float:
    """K-recall@k (Section 5 metrics): mean over queries of |S cap G_K| / K."""
    return float(np.mean([len(set(f.tolist()) & set(g[:K].tolist())) / K
                          for f, g in zip(found, truth)]))


# ============================================================================ loss / gradient
def loss_pairwise(A, B, Q, Xc_list, n_pairs: float | None = None):
    """The LeanVec loss of Problem 3 summed over clusters: sum over q and x in X_c of
    (<A_c q, B_c x> - <q, x>)^2, divided by n_pairs (default m * sum |X_c|).
    Returns (loss, dA, dB) in float64."""
    Q64 = np.asarray(Q, np.float64)
    N = n_pairs if n_pairs is not None else Q64.shape[0] * sum(x.shape[0] for x in Xc_list)
    L = 0.0
    dA = np.zeros_like(np.asarray(A, np.float64))
    dB = np.zeros_like(dA)
    for c, Xc in enumerate(Xc_list):
        Xc = np.asarray(Xc, np.float64)
        if Xc.shape[0] == 0:
            continue
        Ac = np.asarray(A[c], np.float64)
        Bc = np.asarray(B[c], np.float64)
        R = (Q64 @ Ac.T) @ (Xc @ Bc.T).T - Q64 @ Xc.T          # m x n_c residuals
        L += np.sum(R * R)
        dA[c] = 2.0 * Bc @ Xc.T @ R.T @ Q64
        dB[c] = 2.0 * Ac @ Q64.T @ R @ Xc
    return L / N, dA / N, dB / N


def loss_gram(A, B, KQ_sum, KX_sum, n_pairs: float):
    """The same loss through the rewrite of Eq. 5: with M_c = A_c^T B_c - I,
    L = sum_c <K_Q M_c K_{X_c}, M_c>_F / N, dL/dA_c = 2 B_c K_{X_c} M_c^T K_Q / N,
    dL/dB_c = 2 A_c K_Q M_c K_{X_c} / N (K_Q and K_{X_c} are sums)."""
    C, d, D = np.shape(A)
    I = np.eye(D)
    L = 0.0
    dA = np.zeros((C, d, D))
    dB = np.zeros((C, d, D))
    for c in range(C):
        Ac = np.asarray(A[c], np.float64)
        Bc = np.asarray(B[c], np.float64)
        M = Ac.T @ Bc - I
        KQM = KQ_sum @ M
        L += np.sum((KQM @ KX_sum[c]) * M)
        dA[c] = 2.0 * Bc @ KX_sum[c] @ M.T @ KQ_sum
        dB[c] = 2.0 * Ac @ KQM @ KX_sum[c]
    return L / n_pairs, dA / n_pairs, dB / n_pairs
