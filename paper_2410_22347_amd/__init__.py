"""GleanVec / LeanVec-Sphering on MI355X (gfx950): Python binding.

A thin ctypes layer over ``libgleanvec.so`` (C ABI in ``include/gleanvec.h``).
It only marshals arguments: torch tensors supply device memory and the
current HIP stream; every step of fit, encode and search runs in the
library's HIP kernels.  Importing this package fails loudly when the library
has not been built (``python -m paper_2410_22347_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgleanvec.so")

FP32, FP16, BF16, FP8 = 0, 1, 2, 3
FORMATS = {"fp32": FP32, "fp16": FP16, "bf16": BF16, "fp8": FP8}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}

_STATUS = {0: "GV_OK", -1: "GV_EINVAL", -2: "GV_ENOMEM", -3: "GV_EDEVICE", -4: "GV_ENOTFIT",
           -5: "GV_ENONFINITE", -6: "GV_EUNSUPPORTED", -7: "GV_ENOCONV"}

EXPORTED = [
    "gv_status_string", "gv_last_error", "gv_fit", "gv_model_import", "gv_model_shape",
    "gv_model_export", "gv_model_stats", "gv_model_destroy", "gv_encode", "gv_index_shape",
    "gv_index_export", "gv_index_destroy", "gv_search", "gv_project", "gv_score_topk",
    "gv_rerank", "gv_search_tuning", "gv_search_optimism", "gv_debug_fail_alloc", "gv_debug_allocs_pending",
    "gv_host_eigh", "gv_profile_enable", "gv_profile_read",
    "gv_padded_dim", "gv_tags", "gv_moments", "gv_loss_grad", "gv_search_batched", "gv_batch_release",
    "gv_search_flex", "gv_project_flex", "gv_score_topk_flex", "gv_rerank_stored", "gv_augment",
    "gv_moments_update", "gv_fit_from_stats", "gv_batch_counts", "gv_eig_step_limit",
    "gv_model_save", "gv_model_load", "gv_model_file_info", "gv_model_sphering", "gv_scan_plan",
    "gv_search_noalloc", "gv_search_noalloc_capacity", "gv_index_reproject", "gv_index_rows", "gv_search_lazy",
    "gv_autotune", "gv_tuning_table_save", "gv_tuning_table_load", "gv_tuning_lookup", "gv_tuning_table_clear",
]


class GleanVecError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2410_22347_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64


class _FitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("kmeans_sample", ctypes.c_int64), ("init_centroids", _vp)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("gv_status_string", [ctypes.c_int], ctypes.c_char_p)
_sig("gv_last_error", [], ctypes.c_char_p)
_sig("gv_fit", [_vp, _i64, _vp, _i64, _i32, _i32, _i32, _u64, ctypes.POINTER(_FitOpts), _vp, ctypes.POINTER(_vp)])
_sig("gv_model_import", [_vp, _vp, _vp, _i32, _i32, _i32, ctypes.POINTER(_vp)])
_sig("gv_model_shape", [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
_sig("gv_model_export", [_vp, _vp, _vp, _vp])
_sig("gv_model_stats", [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32)])
_sig("gv_model_destroy", [_vp], None)
_sig("gv_encode", [_vp, _vp, _i64, ctypes.c_int, _i32, _vp, ctypes.POINTER(_vp)])
_sig("gv_index_shape", [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                        ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
_sig("gv_index_export", [_vp, _vp, _vp, _vp, _vp, _vp])
_sig("gv_index_destroy", [_vp], None)
_sig("gv_index_reproject", [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.c_int, _vp, ctypes.POINTER(_vp)])
_sig("gv_index_rows", [_vp, ctypes.POINTER(_i64)])
_sig("gv_search", [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp])
_sig("gv_search_noalloc", [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp])
_sig("gv_search_lazy", [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp])
_sig("gv_search_noalloc_capacity", [], _i64)
_sig("gv_project", [_vp, ctypes.c_int, _vp, _i64, _vp, _vp, _vp, _vp])
_sig("gv_score_topk", [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp])
_sig("gv_rerank", [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp])
_sig("gv_search_tuning", [_i32, _i32, _i32])
_sig("gv_search_optimism", [_i32])
_sig("gv_debug_fail_alloc", [_i32])
_sig("gv_debug_allocs_pending", [], _i32)
_sig("gv_augment", [_vp, _i64, _i32, _i32, _vp, _vp])
_sig("gv_moments_update", [_vp, _i64, _i32, _vp, _i32, _i32, _vp, _vp])
_sig("gv_fit_from_stats", [_vp, _vp, ctypes.c_double, _vp, _vp, _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)])
_sig("gv_search_flex", [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp])
_sig("gv_project_flex", [_vp, ctypes.c_int, _vp, _i64, _i32, _vp, _vp, _vp, _vp])
_sig("gv_score_topk_flex", [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp])
_sig("gv_rerank_stored", [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp])
_sig("gv_padded_dim", [_i32], _i32)
_sig("gv_host_eigh", [_i32, _vp, _vp, _vp])
_sig("gv_eig_step_limit", [_i32])
_sig("gv_model_save", [_vp, ctypes.c_char_p])
_sig("gv_model_load", [ctypes.c_char_p, ctypes.POINTER(_vp)])
_sig("gv_model_file_info", [ctypes.c_char_p, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                            ctypes.POINTER(_i32)])
_sig("gv_model_sphering", [_vp, _vp, _vp, _vp])
_sig("gv_scan_plan", [_i64, _i64, _i32, ctypes.c_int, _i32, _i32, _i64, _i32, _vp, _i32, ctypes.POINTER(_i32),
                      ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("gv_profile_enable", [_i32])
_sig("gv_tags", [_vp, _vp, _i64, _vp, _vp])
_sig("gv_search_batched", [_i32, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp])
_sig("gv_batch_release", [], None)
_sig("gv_batch_counts", [ctypes.POINTER(_i64), ctypes.POINTER(_i64)], None)
_sig("gv_moments", [_vp, _i64, _i32, _vp, _i32, _vp, _vp])
_sig("gv_loss_grad", [_i32, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp])
_sig("gv_profile_read", [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(_i64)])


class _TuneResult(ctypes.Structure):
    _fields_ = [("splits", ctypes.c_int32), ("qpw", ctypes.c_int32), ("cap", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_automatic", ctypes.c_double), ("candidates", ctypes.c_int32)]


_sig("gv_autotune", [_vp, _vp, _vp, _i64, _i32, _i32, _i32, ctypes.POINTER(_TuneResult), _vp])
_sig("gv_tuning_table_save", [ctypes.c_char_p])
_sig("gv_tuning_table_load", [ctypes.c_char_p])
_sig("gv_tuning_lookup", [_i32, _i32, _i64, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
_sig("gv_tuning_table_clear", [], None)


def _check(status: int, where: str):
    if status != 0:
        raise GleanVecError(status, where, (_lib.gv_last_error() or b"").decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2):
        raise ValueError("expected a contiguous 2-D float32 CUDA tensor")
    return t


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Model:
    """Landmarks mu_c and projections A_c, B_c (owned by the library)."""

    def __init__(self, handle):
        self._h = handle
        C, d, D = _i32(), _i32(), _i32()
        _check(_lib.gv_model_shape(self._h, ctypes.byref(C), ctypes.byref(d), ctypes.byref(D)), "gv_model_shape")
        self.C, self.d, self.D = C.value, d.value, D.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gv_model_destroy(self._h)
            self._h = None

    def export(self):
        mu = np.empty((self.C, self.D))
        A = np.empty((self.C, self.d, self.D))
        B = np.empty((self.C, self.d, self.D))
        _check(_lib.gv_model_export(self._h, _np_ptr(mu), _np_ptr(A), _np_ptr(B)), "gv_model_export")
        return mu, A, B

    def stats(self):
        C, D = self.C, self.D
        KQ = np.empty((D, D)); KX = np.empty((C, D, D)); lamQ = np.empty(D); lamc = np.empty((C, D))
        counts = np.empty(C, np.int64); fb = np.empty(C, np.uint8); it = _i32()
        _check(_lib.gv_model_stats(self._h, _np_ptr(KQ), _np_ptr(KX), _np_ptr(lamQ), _np_ptr(lamc),
                                   _np_ptr(counts), _np_ptr(fb), ctypes.byref(it)), "gv_model_stats")
        return dict(KQ=KQ, KX=KX, lam_Q=lamQ, lam_c=lamc, counts=counts, fallback=fb.astype(bool),
                    iters=it.value)

    def sphering(self):
        """(W, W+, P) of a fitted model: D x D, D x D, C x d x D."""
        W = np.empty((self.D, self.D)); Wp = np.empty((self.D, self.D)); P = np.empty((self.C, self.d, self.D))
        _check(_lib.gv_model_sphering(self._h, _np_ptr(W), _np_ptr(Wp), _np_ptr(P)), "gv_model_sphering")
        return W, Wp, P

    def save(self, path: str):
        """Write the model to a file (gv_model_save)."""
        _check(_lib.gv_model_save(self._h, os.fsencode(path)), "gv_model_save")


def model_load(path: str) -> Model:
    """A model read from a file written by Model.save (gv_model_load)."""
    h = _vp()
    _check(_lib.gv_model_load(os.fsencode(path), ctypes.byref(h)), "gv_model_load")
    return Model(h)


def model_file_info(path: str):
    """Validate a model file without the device: (C, d, D, has_stats)."""
    C, d, D, st = _i32(), _i32(), _i32(), _i32()
    _check(_lib.gv_model_file_info(os.fsencode(path), ctypes.byref(C), ctypes.byref(d), ctypes.byref(D),
                                   ctypes.byref(st)), "gv_model_file_info")
    return C.value, d.value, D.value, bool(st.value)


class Index:
    """Grouped, quantised reduced database plus the FP32 vectors for the rerank."""

    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep          # a borrowed X must outlive the index
        n, C, d, dp, f = _i64(), _i32(), _i32(), _i32(), _i32()
        _check(_lib.gv_index_shape(self._h, ctypes.byref(n), ctypes.byref(C), ctypes.byref(d), ctypes.byref(dp),
                                   ctypes.byref(f)), "gv_index_shape")
        self.n, self.C, self.d, self.d_pad, self.fmt = n.value, C.value, d.value, dp.value, f.value
        rows = _i64()
        _check(_lib.gv_index_rows(self._h, ctypes.byref(rows)), "gv_index_rows")
        self.rows = rows.value   # stored vectors (n minus removed ids)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gv_index_destroy(self._h)
            self._h = None

    def export(self):
        eb = {FP32: 4, FP16: 2, BF16: 2, FP8: 1}[self.fmt]
        dt = {4: np.uint32, 2: np.uint16, 1: np.uint8}[eb]
        tags = np.empty(self.n, np.uint8)
        off = np.empty(self.C + 1, np.int64)
        ids = np.empty(self.rows, np.int32)
        xlow = np.empty((self.rows, self.d_pad), dt)
        scale = np.empty(self.C, np.float32)
        _check(_lib.gv_index_export(self._h, _np_ptr(tags), _np_ptr(off), _np_ptr(ids), _np_ptr(xlow),
                                    _np_ptr(scale)), "gv_index_export")
        return dict(tags=tags, offsets=off, ids=ids, xlow=xlow, scale=scale)


def fit(X_learn, Q_learn, d: int, C: int, seed: int, max_iter: int = 0, kmeans_sample: int = 0,
        init_centroids=None) -> Model:
    """GleanVec learning (Algorithm 5) on the current device."""
    _dev_f32(X_learn); _dev_f32(Q_learn)
    opts = _FitOpts(max_iter, kmeans_sample, None)
    keep = None
    if init_centroids is not None:
        keep = np.ascontiguousarray(init_centroids, np.float64)
        opts.init_centroids = keep.ctypes.data
    h = _vp()
    _check(_lib.gv_fit(_ptr(X_learn), X_learn.shape[0], _ptr(Q_learn), Q_learn.shape[0], X_learn.shape[1], d, C,
                       seed & ((1 << 64) - 1), ctypes.byref(opts), _stream(), ctypes.byref(h)), "gv_fit")
    return Model(h)


def model_import(mu, A, B) -> Model:
    mu = np.ascontiguousarray(mu, np.float64)
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    C, d, D = A.shape
    h = _vp()
    _check(_lib.gv_model_import(_np_ptr(mu), _np_ptr(A), _np_ptr(B), C, d, D, ctypes.byref(h)), "gv_model_import")
    return Model(h)


def encode(model: Model, X, fmt, copy_X=False) -> Index:
    """Index build.  copy_X: False borrows X (kept alive by the Index), True copies
    it, "none" keeps no full-dimension vectors (rerank from the stored ones)."""
    _dev_f32(X)
    f = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    mode = 2 if copy_X == "none" else (1 if copy_X else 0)
    h = _vp()
    _check(_lib.gv_encode(model._h, _ptr(X), X.shape[0], f, mode, _stream(), ctypes.byref(h)), "gv_encode")
    return Index(h, keep=X if mode == 0 else None)


def search(model: Model, index: Index, Q, k: int, kappa: int, with_scores: bool = True):
    """Multi-step search; returns (ids [m, k] int32, scores [m, k] float32 or None)."""
    import torch
    _dev_f32(Q)
    m = Q.shape[0]
    ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=Q.device) if with_scores else None
    _check(_lib.gv_search(model._h, index._h, _ptr(Q), m, k, kappa, _ptr(ids), _ptr(sc), _stream()), "gv_search")
    return ids, sc


def index_reproject(old_model: Model, new_model: Model, index: Index, keep=None, X_new=None, fmt=None) -> Index:
    """gv_index_reproject: the index's stored vectors carried to new_model's
    projections without X (Section 3, streaming), plus inserted vectors X_new
    (ids index.n ...), minus the ids whose keep flag (uint8 CUDA tensor, one per
    id) is zero.  The result keeps no full-dimension vectors."""
    import torch
    f = FORMATS[fmt] if isinstance(fmt, str) else (index.fmt if fmt is None else fmt)
    if keep is not None and not (keep.is_cuda and keep.dtype == torch.uint8 and keep.numel() == index.n
                                 and keep.is_contiguous()):
        raise ValueError("keep must be a contiguous uint8 CUDA tensor with one flag per id")
    n_new = 0
    if X_new is not None:
        _dev_f32(X_new)
        n_new = X_new.shape[0]
    h = _vp()
    _check(_lib.gv_index_reproject(old_model._h, new_model._h, index._h, _ptr(keep), _ptr(X_new), n_new, f,
                                   _stream(), ctypes.byref(h)), "gv_index_reproject")
    return Index(h)


def search_noalloc_into(model: Model, index: Index, Q, k: int, kappa: int, out_ids, out_scores=None):
    """gv_search_noalloc: the search into caller-given outputs, with no device
    allocation inside the library (its scratch is a fixed per-device array)."""
    _dev_f32(Q)
    m = Q.shape[0]
    if tuple(out_ids.shape) != (m, k) or (out_scores is not None and tuple(out_scores.shape) != (m, k)):
        raise ValueError("outputs must be m x k")
    _check(_lib.gv_search_noalloc(model._h, index._h, _ptr(Q), m, k, kappa, _ptr(out_ids), _ptr(out_scores),
                                  _stream()), "gv_search_noalloc")
    return out_ids, out_scores


def search_noalloc_capacity() -> int:
    return int(_lib.gv_search_noalloc_capacity())


def search_lazy(model: Model, index: Index, Q, k: int, kappa: int):
    """The search with the lazy inner product of Algorithm 3 (gv_search_lazy)."""
    import torch
    _dev_f32(Q)
    m = Q.shape[0]
    ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    _check(_lib.gv_search_lazy(model._h, index._h, _ptr(Q), m, k, kappa, _ptr(ids), _ptr(sc), _stream()),
           "gv_search_lazy")
    return ids, sc


def augment(V, kind: str):
    """Euclidean adaptation: [v, -||v||^2 / 2] (kind "database") or [v, 1] ("query")."""
    import torch
    _dev_f32(V)
    n, D = V.shape
    out = torch.empty((n, D + 1), dtype=torch.float32, device=V.device)
    _check(_lib.gv_augment(_ptr(V), n, D, {"database": 0, "query": 1}[kind], _ptr(out), _stream()), "gv_augment")
    return out


RERANK = {"full": 0, "stored": 1}


def search_flex(model: Model, index: Index, Q, k: int, kappa: int, d_search: int, rerank: str = "full",
                with_scores: bool = True):
    """Search on the leading d_search coordinates (Section 3.3); rerank "full" (exact,
    from X) or "stored" (from the stored vectors).  Returns (ids, scores or None)."""
    import torch
    _dev_f32(Q)
    m = Q.shape[0]
    ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=Q.device) if with_scores else None
    _check(_lib.gv_search_flex(model._h, index._h, _ptr(Q), m, k, kappa, d_search, RERANK[rerank], _ptr(ids),
                               _ptr(sc), _stream()), "gv_search_flex")
    return ids, sc


def project_flex(model: Model, fmt, Q, d_search: int):
    """Stage S1 of search_flex: (q_c [m, C, d_pad] f32 over all d rows, t [m, C],
    qhat [m, C, padded_dim(d_search)] raw format of the first d_search values)."""
    import torch
    _dev_f32(Q)
    f = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    m = Q.shape[0]
    qc = torch.empty((m, model.C, padded_dim(model.d)), dtype=torch.float32, device=Q.device)
    t = torch.empty((m, model.C), dtype=torch.float32, device=Q.device)
    qhat = torch.empty((m, model.C, padded_dim(d_search)), dtype=_view_dtype(f), device=Q.device)
    _check(_lib.gv_project_flex(model._h, f, _ptr(Q), m, d_search, _ptr(qc), _ptr(t), _ptr(qhat), _stream()),
           "gv_project_flex")
    return qc, t, qhat


def score_topk_flex(index: Index, qhat, t, d_search: int, kappa: int):
    """Stages S2 + S3 on the leading d_search coordinates: (cand_ids, cand_scores)."""
    import torch
    m = t.shape[0]
    ids = torch.empty((m, kappa), dtype=torch.int32, device=t.device)
    sc = torch.empty((m, kappa), dtype=torch.float32, device=t.device)
    _check(_lib.gv_score_topk_flex(index._h, _ptr(qhat), _ptr(t), m, d_search, kappa, _ptr(ids), _ptr(sc),
                                   _stream()), "gv_score_topk_flex")
    return ids, sc


def rerank_stored(index: Index, qc, cand_ids, k: int):
    """Stage S4 from the stored vectors: (ids [m, k] int32, scores [m, k] f32)."""
    import torch
    m, kappa = cand_ids.shape
    ids = torch.empty((m, k), dtype=torch.int32, device=qc.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=qc.device)
    _check(_lib.gv_rerank_stored(index._h, _ptr(qc), m, _ptr(cand_ids), kappa, k, _ptr(ids), _ptr(sc), _stream()),
           "gv_rerank_stored")
    return ids, sc


def _view_dtype(fmt):
    """Element type of the query views that meet storage format fmt (FP8 storage
    meets FP16 views)."""
    import torch
    return {FP32: torch.float32, FP16: torch.int16, BF16: torch.int16, FP8: torch.int16}[fmt]


def project(model: Model, fmt, Q, want_qc: bool = True):
    """Stage S1: returns (q_c [m, C, d_pad] f32 or None, t [m, C] f32, qhat [m, C, d_pad] raw format)."""
    import torch
    _dev_f32(Q)
    f = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    m = Q.shape[0]
    dp = padded_dim(model.d)
    qc = torch.empty((m, model.C, dp), dtype=torch.float32, device=Q.device) if want_qc else None
    t = torch.empty((m, model.C), dtype=torch.float32, device=Q.device)
    qhat = torch.empty((m, model.C, dp), dtype=_view_dtype(f), device=Q.device)
    _check(_lib.gv_project(model._h, f, _ptr(Q), m, _ptr(qc), _ptr(t), _ptr(qhat), _stream()), "gv_project")
    return qc, t, qhat


def score_topk(index: Index, qhat, t, kappa: int):
    """Stages S2 + S3: returns (cand_ids [m, kappa] int32, cand_scores [m, kappa] f32)."""
    import torch
    m = t.shape[0]
    ids = torch.empty((m, kappa), dtype=torch.int32, device=t.device)
    sc = torch.empty((m, kappa), dtype=torch.float32, device=t.device)
    _check(_lib.gv_score_topk(index._h, _ptr(qhat), _ptr(t), m, kappa, _ptr(ids), _ptr(sc), _stream()),
           "gv_score_topk")
    return ids, sc


def rerank(index: Index, Q, cand_ids, k: int):
    """Stage S4: returns (ids [m, k] int32, scores [m, k] f32)."""
    import torch
    _dev_f32(Q)
    m, kappa = cand_ids.shape
    ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    _check(_lib.gv_rerank(index._h, _ptr(Q), m, _ptr(cand_ids), kappa, k, _ptr(ids), _ptr(sc), _stream()),
           "gv_rerank")
    return ids, sc


def search_tuning(splits: int = 0, qpw: int = 0, cap: int = 0):
    _check(_lib.gv_search_tuning(splits, qpw, cap), "gv_search_tuning")


def debug_fail_alloc(after: int = -1):
    """gv_debug_fail_alloc: the library's (after + 1)-th device allocation from now
    fails as out of memory (-1: off).  For tests."""
    _check(_lib.gv_debug_fail_alloc(after), "gv_debug_fail_alloc")


def debug_allocs_pending() -> int:
    return int(_lib.gv_debug_allocs_pending())


def search_optimism(rank: int = 0):
    """gv_search_optimism: seed rank of the full scan (0 automatic, -1 the exact
    kappa-th best of the sample, k > 0 the k-th best; results do not change)."""
    _check(_lib.gv_search_optimism(rank), "gv_search_optimism")


def autotune(model: Model, index: Index, Q, k: int, kappa: int, reps: int = 3):
    """gv_autotune: time candidate launch shapes for this search's shape class and
    keep the fastest in the process's table; returns the choice as a dict."""
    _dev_f32(Q)
    r = _TuneResult()
    _check(_lib.gv_autotune(model._h, index._h, _ptr(Q), Q.shape[0], k, kappa, reps, ctypes.byref(r), _stream()),
           "gv_autotune")
    return dict(splits=r.splits, qpw=r.qpw, cap=r.cap, ms=r.ms, ms_automatic=r.ms_automatic,
                candidates=r.candidates)


def tuning_table_save(path: str):
    _check(_lib.gv_tuning_table_save(os.fsencode(path)), "gv_tuning_table_save")


def tuning_table_load(path: str):
    _check(_lib.gv_tuning_table_load(os.fsencode(path)), "gv_tuning_table_load")


def tuning_lookup(fmt, d_pad: int, m: int, n_rows: int):
    """The table's (splits, qpw, cap) for a shape class, or None."""
    f = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    sp, qpw, cap = _i32(), _i32(), _i32()
    st = _lib.gv_tuning_lookup(f, d_pad, m, n_rows, ctypes.byref(sp), ctypes.byref(qpw), ctypes.byref(cap))
    return None if st != 0 else (sp.value, qpw.value, cap.value)


def tuning_table_clear():
    _lib.gv_tuning_table_clear()


def padded_dim(d: int) -> int:
    return int(_lib.gv_padded_dim(d))


def host_eigh(A):
    """The library's host FP64 symmetric eigensolver (decreasing eigenvalues, rows = vectors)."""
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    lam = np.empty(n)
    Vt = np.empty((n, n))
    _check(_lib.gv_host_eigh(n, _np_ptr(A), _np_ptr(lam), _np_ptr(Vt)), "gv_host_eigh")
    return lam, Vt


def eig_step_limit(max_steps: int = 0):
    """QR step budget of one host eigendecomposition (0: the default, 60 x order)."""
    _check(_lib.gv_eig_step_limit(int(max_steps)), "gv_eig_step_limit")


def profile_enable(on: bool = True):
    _check(_lib.gv_profile_enable(1 if on else 0), "gv_profile_enable")


def profile_read():
    """(ms_score, n_score, ms_merge, n_merge) since the last read; waits for the events."""
    a, c = ctypes.c_double(), ctypes.c_double()
    b, d = _i64(), _i64()
    _check(_lib.gv_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
           "gv_profile_read")
    return a.value, b.value, c.value, d.value


def search_batched(models, indexes, Qs, k: int, kappa: int, out=None):
    """Algorithm 1 for several collections in one graph launch (gv_search_batched).
    Qs: list of float32 CUDA tensors (m_i x D_i).  out: optional list of
    (ids, scores) tensors from a previous call with the same shapes; passing them
    back with the same query tensors replays the captured graph.
    Returns the list of (ids, scores)."""
    import torch
    n = len(models)
    if not (len(indexes) == n and len(Qs) == n):
        raise ValueError("search_batched: models, indexes and Qs differ in length")
    if out is None:
        out = [(torch.empty((Q.shape[0], k), dtype=torch.int32, device=Q.device),
                torch.empty((Q.shape[0], k), dtype=torch.float32, device=Q.device)) for Q in Qs]
    for Q, md, (ids, sc) in zip(Qs, models, out):
        _dev_f32(Q)
        if Q.shape[1] != md.D or ids.shape != (Q.shape[0], k) or sc.shape != (Q.shape[0], k):
            raise ValueError("search_batched: query or output shapes differ")
    arr = lambda vals: (ctypes.c_void_p * n)(*vals)
    mh = arr([md._h for md in models])
    ih = arr([ix._h for ix in indexes])
    qp = arr([Q.data_ptr() for Q in Qs])
    ms = (ctypes.c_int64 * n)(*[Q.shape[0] for Q in Qs])
    op = arr([o[0].data_ptr() for o in out])
    sp = arr([o[1].data_ptr() for o in out])
    _check(_lib.gv_search_batched(n, mh, ih, qp, ms, k, kappa, op, sp, _stream()), "gv_search_batched")
    return out


def batch_release():
    _lib.gv_batch_release()


def batch_counts():
    """(captures, replays) of gv_search_batched since the library was loaded."""
    c, r = _i64(0), _i64(0)
    _lib.gv_batch_counts(ctypes.byref(c), ctypes.byref(r))
    return c.value, r.value


def tags(model: Model, X):
    """Cluster tags arg-max_c <x, mu_c> (FP64, lowest c on ties) as a uint8 CUDA tensor."""
    import torch
    X = _dev_f32(X)
    if X.shape[1] != model.D:
        raise ValueError("X has the wrong dimension")
    out = torch.empty((X.shape[0],), dtype=torch.uint8, device=X.device)
    _check(_lib.gv_tags(model._h, _ptr(X), X.shape[0], _ptr(out), _stream()), "gv_tags")
    return out


def moments(V, tags_=None, C: int = 1):
    """Uncentered second-moment sums K[c] = sum_{tag == c} v v^T (FP64, C x D x D)."""
    import torch
    V = _dev_f32(V)
    if tags_ is not None and not (tags_.is_cuda and tags_.dtype == torch.uint8 and tags_.is_contiguous()
                                  and tags_.shape == (V.shape[0],)):
        raise ValueError("tags must be a contiguous uint8 CUDA tensor with one entry per row")
    D = V.shape[1]
    K = torch.empty((C, D, D), dtype=torch.float64, device=V.device)
    _check(_lib.gv_moments(_ptr(V), V.shape[0], D, _ptr(tags_), C, _ptr(K), _stream()), "gv_moments")
    return K


def moments_update(K, V, tags_=None, sign: int = 1):
    """Streaming update in place: K[c] += sign * sum_{tag == c} v v^T (sign +1 insert, -1 remove)."""
    import torch
    V = _dev_f32(V)
    if tags_ is not None and not (tags_.is_cuda and tags_.dtype == torch.uint8 and tags_.is_contiguous()
                                  and tags_.shape == (V.shape[0],)):
        raise ValueError("tags must be a contiguous uint8 CUDA tensor with one entry per row")
    if not (K.is_cuda and K.dtype == torch.float64 and K.is_contiguous() and K.dim() == 3):
        raise ValueError("K must be a contiguous C x D x D float64 CUDA tensor")
    _check(_lib.gv_moments_update(_ptr(V), V.shape[0], V.shape[1], _ptr(tags_), K.shape[0], sign, _ptr(K),
                                  _stream()), "gv_moments_update")
    return K


def fit_from_stats(mu, KQ, m_q: float, KX, counts, d: int) -> Model:
    """Projections recomputed from kept statistics (streaming updates): mu host C x D,
    KQ device D x D sum over m_q queries, KX device C x D x D sums, counts host C."""
    import torch
    mu = np.ascontiguousarray(mu, np.float64)
    counts = np.ascontiguousarray(counts, np.int64)
    C, D = mu.shape
    for t, shape in ((KQ, (D, D)), (KX, (C, D, D))):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"statistics must be contiguous float64 CUDA tensors of shape {shape}")
    h = _vp()
    _check(_lib.gv_fit_from_stats(_np_ptr(mu), _ptr(KQ), float(m_q), _ptr(KX), _np_ptr(counts), C, d, D, _stream(),
                                  ctypes.byref(h)), "gv_fit_from_stats")
    return Model(h)


def loss_grad(A, B, KQ, KX, n_pairs: float, grads: bool = True):
    """(loss, dA, dB) of the inner-product approximation loss (Gram form); see gv_loss_grad.
    A, B: float32 CUDA (C, d, D); KQ: float64 (D, D); KX: float64 (C, D, D)."""
    import torch
    for t, dt, nd in ((A, torch.float32, 3), (B, torch.float32, 3), (KQ, torch.float64, 2), (KX, torch.float64, 3)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == nd):
            raise ValueError("loss_grad: expected contiguous CUDA tensors A, B (float32, C x d x D), "
                             "KQ (float64, D x D), KX (float64, C x D x D)")
    C, d, D = A.shape
    if B.shape != A.shape or KQ.shape != (D, D) or KX.shape != (C, D, D):
        raise ValueError("loss_grad: shapes differ")
    loss = torch.empty((), dtype=torch.float64, device=A.device)
    dA = torch.empty_like(A) if grads else None
    dB = torch.empty_like(B) if grads else None
    _check(_lib.gv_loss_grad(C, d, D, _ptr(A), _ptr(B), _ptr(KQ), _ptr(KX), float(n_pairs), _ptr(loss), _ptr(dA),
                             _ptr(dB), _stream()), "gv_loss_grad")
    return loss, dA, dB


def _make_loss_fn():
    import torch

    class GleanLoss(torch.autograd.Function):
        """torch.autograd.Function over gv_loss_grad: forward returns the loss
        (float64 scalar); the gradient with respect to A and B comes from the
        same library call, scaled by the incoming gradient."""

        @staticmethod
        def forward(ctx, A, B, KQ, KX, n_pairs):
            loss, dA, dB = loss_grad(A.detach().contiguous(), B.detach().contiguous(), KQ, KX, n_pairs)
            ctx.save_for_backward(dA, dB)
            return loss

        @staticmethod
        def backward(ctx, g):
            dA, dB = ctx.saved_tensors
            return (g * dA).to(dA.dtype), (g * dB).to(dB.dtype), None, None, None

    return GleanLoss


_loss_fn = None


def gleanvec_loss(A, B, KQ, KX, n_pairs: float):
    """Differentiable loss of the per-cluster projections A, B (see GleanLoss)."""
    global _loss_fn
    if _loss_fn is None:
        _loss_fn = _make_loss_fn()
    return _loss_fn.apply(A, B, KQ, KX, n_pairs)


def status_string(code: int) -> str:
    return _lib.gv_status_string(code).decode()
