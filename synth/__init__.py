"""Seeded synthetic inputs shared by the oracle-side tests and the device path.

This module only *draws data*: Gaussian mixtures with decaying spectra and
out-of-distribution (OOD) query laws.  It holds none of the search method's
arithmetic (no projections, no clustering, no scoring), so the oracle and the
HIP path can both consume its output without sharing any method code.

Recipe (stand-in for the paper's real embedding datasets, Table 1, which are
not available here): FP32 vectors compared by inner product, separate learn and
test query sets, OOD queries (shifted means and rotated covariance, Section 2).

* ``linear`` law (one component, zero mean): x = R_x (lambda^(1/2) * z) with
  lambda_i = 1/i and a Haar rotation R_x; queries use an independent Haar R_q.
* ``mixture`` law with J components: mean mu_j = g/|g|; covariance
  R_j diag(lambda^(j)) R_j^T with lambda^(j)_i = i^(-alpha_j) / sum_l l^(-alpha_j)
  (unit trace) and alpha_j = 0.75 + 0.5 j/(J-1); uniform weights.  OOD queries of
  component j have mean mu_j + 0.5 u_j (u_j uniform on the sphere) and
  covariance G Sigma_j G^T with one shared Haar rotation G.

Every stream is ``numpy.random.default_rng(SeedSequence([ROOT, cfg, stream,
chunk]))``; the database is drawn in chunks of 2**16 rows so any chunk can be
regenerated on its own.  A second, device-side backend (``*_torch``) draws the
bulk Gaussians with a seeded ``torch.Generator`` on the GPU for workloads too
large to draw on the host; the geometry (means, rotations) is always drawn by
numpy so both backends share it.
"""
from __future__ import annotations

import dataclasses
import numpy as np

ROOT = 0x241022347
CHUNK = 1 << 16

# stream ids
S_GEOM, S_DB, S_QLEARN, S_QTEST, S_SAMPLE, S_SEED, S_QTRAIN = range(7)


def rng_for(cfg: int, stream: int, chunk: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT, cfg, stream, chunk]))


def haar(rng: np.random.Generator, D: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian, signs fixed by diag R)."""
    g = rng.standard_normal((D, D))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


@dataclasses.dataclass
class Geometry:
    law: str            # "linear" or "mixture"
    cfg: int
    D: int
    J: int
    means: np.ndarray   # J x D  (zeros for the linear law)
    rots: np.ndarray    # J x D x D  data rotations R_j
    sqrt_lam: np.ndarray  # J x D  standard deviations along R_j's columns
    q_means: np.ndarray   # J x D  query means
    q_rot: np.ndarray     # D x D  shared query rotation (G, or R_q for linear)


def make_geometry(cfg: int, D: int, J: int, law: str = "mixture") -> Geometry:
    rng = rng_for(cfg, S_GEOM)
    if law == "linear":
        lam = 1.0 / np.arange(1, D + 1, dtype=np.float64)
        R = haar(rng, D)
        G = haar(rng, D)
        return Geometry(law, cfg, D, 1, np.zeros((1, D)), R[None], np.sqrt(lam)[None],
                        np.zeros((1, D)), G)
    means = np.empty((J, D))
    rots = np.empty((J, D, D))
    sl = np.empty((J, D))
    i = np.arange(1, D + 1, dtype=np.float64)
    for j in range(J):
        g = rng.standard_normal(D)
        means[j] = g / np.linalg.norm(g)
        rots[j] = haar(rng, D)
        alpha = 0.75 + 0.5 * (j / (J - 1) if J > 1 else 0.0)
        lam = i ** (-alpha)
        sl[j] = np.sqrt(lam / lam.sum())
    u = rng.standard_normal((J, D))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q_means = means + 0.5 * u
    G = haar(rng, D)
    return Geometry(law, cfg, D, J, means, rots, sl, q_means, G)


def _draw(geom: Geometry, rng: np.random.Generator, n: int, queries: bool) -> np.ndarray:
    comp = rng.integers(0, geom.J, size=n)
    z = rng.standard_normal((n, geom.D))
    out = np.empty((n, geom.D))
    for j in range(geom.J):
        sel = np.nonzero(comp == j)[0]
        if sel.size == 0:
            continue
        w = z[sel] * geom.sqrt_lam[j]
        if geom.law == "linear":
            y = w @ (geom.q_rot if queries else geom.rots[0]).T
        else:
            y = w @ geom.rots[j].T
            if queries:
                y = y @ geom.q_rot.T
        out[sel] = y + (geom.q_means[j] if queries else geom.means[j])
    return out.astype(np.float32)


def database(geom: Geometry, n: int, start: int = 0) -> np.ndarray:
    """Rows [start, start+n) of the database, FP32, drawn chunk by chunk."""
    rows = []
    c0, c1 = start // CHUNK, (start + n - 1) // CHUNK if n > 0 else start // CHUNK - 1
    for c in range(c0, c1 + 1):
        blk = _draw(geom, rng_for(geom.cfg, S_DB, c), CHUNK, queries=False)
        lo = max(start, c * CHUNK) - c * CHUNK
        hi = min(start + n, (c + 1) * CHUNK) - c * CHUNK
        rows.append(blk[lo:hi])
    if not rows:
        return np.zeros((0, geom.D), np.float32)
    return np.ascontiguousarray(np.concatenate(rows, axis=0))


def queries(geom: Geometry, m: int, stream: int = S_QTEST) -> np.ndarray:
    return _draw(geom, rng_for(geom.cfg, stream), m, queries=True)


# --------------------------------------------------------------------------- device backend

def _torch_seed(cfg: int, stream: int) -> int:
    return int(np.random.SeedSequence([ROOT, cfg, stream, 0xD]).generate_state(1, np.uint64)[0] >> 1)


def draw_torch(geom: Geometry, n: int, stream: int, device, queries_: bool = False,
               block: int = 1 << 20):
    """Draw n FP32 rows on ``device`` (same law as :func:`database` / :func:`queries`,
    different random stream).  Used only for workloads too large for host drawing."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(_torch_seed(geom.cfg, stream))
    D = geom.D
    rots = torch.as_tensor(geom.rots, dtype=torch.float32, device=device)
    sl = torch.as_tensor(geom.sqrt_lam, dtype=torch.float32, device=device)
    mu = torch.as_tensor(geom.q_means if queries_ else geom.means, dtype=torch.float32, device=device)
    G = torch.as_tensor(geom.q_rot, dtype=torch.float32, device=device)
    out = torch.empty((n, D), dtype=torch.float32, device=device)
    for s in range(0, n, block):
        e = min(n, s + block)
        comp = torch.randint(0, geom.J, (e - s,), generator=gen, device=device)
        z = torch.randn((e - s, D), generator=gen, device=device)
        for j in range(geom.J):
            idx = torch.nonzero(comp == j).squeeze(1)
            if idx.numel() == 0:
                continue
            if geom.law == "linear":
                R = G if queries_ else rots[0]
                y = (z[idx] * sl[0]) @ R.T
            else:
                y = (z[idx] * sl[j]) @ rots[j].T
                if queries_:
                    y = y @ G.T
            out[s + idx] = y + mu[j]
        del z, comp
    return out


# --------------------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    cfg: int
    law: str
    D: int
    J: int
    C: int
    d: int
    n: int
    m_learn: int
    m_test: int
    kappa: int
    k: int = 10


WORKLOADS = {
    # LeanVec-Sphering (C = 1), FP32, 1/i spectrum, rotated query law
    "linear-10k-d128": Workload("linear-10k-d128", 1, "linear", 128, 1, 1, 32, 10_000, 10_000, 100, 50),
    # GleanVec C = 16, D = 512 -> 128
    "mix16-1m-d512": Workload("mix16-1m-d512", 2, "mixture", 512, 16, 16, 128, 1_000_000, 10_000, 10_000, 100),
    # GleanVec C = 32, n = 10M, D = 768 -> 160 (shape of RQA-10M-OOD)
    "mix32-10m-d768": Workload("mix32-10m-d768", 3, "mixture", 768, 32, 32, 160, 10_000_000, 10_000, 10_000, 200),
}


def learn_sample_size(n: int) -> int:
    """Rows of the database used as X_learn for the second-moment statistics."""
    return min(n, 1_000_000)


def learn_rows(n: int, n_learn: int, cfg: int) -> np.ndarray:
    """Seeded uniform sample (without replacement, sorted) of database row ids."""
    if n_learn >= n:
        return np.arange(n, dtype=np.int64)
    rng = rng_for(cfg, S_SAMPLE)
    return np.sort(rng.choice(n, size=n_learn, replace=False)).astype(np.int64)


def fit_seed(cfg: int) -> int:
    return int(np.random.SeedSequence([ROOT, cfg, S_SEED]).generate_state(1, np.uint64)[0])


def is_pow2(v: int) -> bool:
    return v > 0 and (v & (v - 1)) == 0


# ------------------------------------------------------------------ batched collections
@dataclasses.dataclass
class Collection:
    cfg: int      # seed domain of this collection's geometry and draws
    n: int
    D: int
    d: int
    C: int
    m: int


def batched_collections(count: int = 64, n_lo: int = 10_000, n_hi: int = 2_000_000, m_hi: int = 4096,
                        dims=(256, 512, 768, 1024), clusters=(4, 16, 32), cfg: int = 4):
    """Uneven collections: n uniform in [n_lo, n_hi], D from dims, d = D/4, C from
    clusters (mixture law with J = C), query batches log-uniform in [1, m_hi]."""
    rng = rng_for(cfg, S_GEOM)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        D = int(rng.choice(dims))
        C = int(rng.choice(clusters))
        m = int(min(m_hi, max(1, round(float(np.exp(rng.uniform(0.0, np.log(m_hi))))))))
        out.append(Collection(1000 * cfg + i, n, D, D // 4, C, m))
    return out
