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


def check_topk_sets(gpu_ids, gpu_scores, ora_scores_by_id, tol_by_id, kappa, what=""):
    """GPU and oracle top-kappa sets may differ only in elements whose oracle score is
    within tolerance of the oracle's kappa-th score; GPU scores must match the
    oracle's within tolerance and be ordered (desc, ties by id)."""
    n = ora_scores_by_id.shape[0]
    ids_all = np.arange(n)
    ora_ids, ora_sc = G.topk(ora_scores_by_id, ids_all, kappa)
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
