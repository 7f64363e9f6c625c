/*
 * gleanvec.h -- C ABI of the MI355X (gfx950) GleanVec / LeanVec-Sphering library.
 *
 * The library implements the data-parallel path of GleanVec (Tepper et al.,
 * "GleanVec: Accelerating vector search with minimalist nonlinear
 * dimensionality reduction", arXiv 2410.22347):
 *
 *   fit     -- learning (Algorithm 5): spherical k-means landmarks
 *              (Appendix A) and one LeanVec-Sphering projection pair per
 *              cluster (Algorithm 2, through the eigendecompositions of the
 *              second-moment statistics of Section 3.2);
 *   encode  -- index build: cluster tags (Eq. 9) and reduced vectors
 *              x_low = B_c x (Eq. 10), grouped by cluster and stored in FP32,
 *              FP16, BF16 or FP8-E4M3 with a per-cluster scale;
 *   search  -- multi-step search (Algorithm 1) with the eager inner product
 *              (Algorithm 4) and a brute-force main step: all views
 *              q_c = A_c q, reduced scores <q_c, x_low_i> (Eq. 11) for every
 *              database vector, the kappa best, and a full-dimension rerank
 *              to the final k.
 *
 * Conventions shared by every call:
 *   - Array arguments marked "device" are device pointers on the current HIP
 *     device (for instance torch tensors' data_ptr()); "host" arrays are
 *     ordinary host memory.  Matrices are row-major and dense.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that take a stream enqueue their device work on it and may return
 *     before it finishes; outputs are valid once the stream has reached that
 *     point.  Calls that return host data synchronise the stream first.
 *   - The caller owns every input and output buffer.  Models and indices own
 *     their device memory until the matching *_destroy call.  Models and
 *     indices are immutable after creation, so concurrent searches on
 *     different streams are safe.
 *   - Every call returns a gv_status; no C++ exception or abort crosses the
 *     ABI.  On error, output handles are set to NULL, and
 *     gv_last_error() returns a thread-local message naming the failure.
 */
#ifndef GLEANVEC_H
#define GLEANVEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GV_OK = 0,
  GV_EINVAL = -1,        /* an argument is out of range or inconsistent */
  GV_ENOMEM = -2,        /* device or host allocation failed */
  GV_EDEVICE = -3,       /* a HIP runtime call failed */
  GV_ENOTFIT = -4,       /* the handle is NULL or was not produced by this library */
  GV_ENONFINITE = -5,    /* an input holds NaN or +-Inf */
  GV_EUNSUPPORTED = -6,  /* valid request that this build does not handle */
  GV_ENOCONV = -7        /* an eigendecomposition of the fit did not converge */
} gv_status;

/* Storage format of the reduced vectors (and of the query views they meet). */
typedef enum {
  GV_FP32 = 0,     /* IEEE binary32, no scaling */
  GV_FP16 = 1,     /* IEEE binary16 */
  GV_BF16 = 2,     /* bfloat16 */
  GV_FP8_E4M3 = 3  /* OCP FP8 E4M3 (e4m3fn: no infinities, max 448) */
} gv_format;

typedef struct gv_model gv_model;
typedef struct gv_index gv_index;

/* Options of gv_fit; a NULL pointer selects every default. */
typedef struct {
  int32_t max_iter;        /* Lloyd steps of spherical k-means, default 50 */
  int64_t kmeans_sample;   /* learn vectors used by k-means, default 100000 (Appendix A) */
  const double* init_centroids; /* host C x D initial landmarks (unit rows) or NULL for k-means++ */
} gv_fit_opts;

/* ------------------------------------------------------------------ errors */

/* Static string naming a status code. */
const char* gv_status_string(gv_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char* gv_last_error(void);

/* ------------------------------------------------------------------ fit */

/*
 * gv_fit -- GleanVec learning, Algorithm 5 of the paper.
 *
 * X_learn  device, n_learn x D FP32: learning database vectors (X_learn).
 * Q_learn  device, m_learn x D FP32: learning queries (Q_learn).
 * d        target dimensionality, 1 <= d <= D.
 * C        number of clusters, 1 <= C <= 255.
 * seed     seed of the SplitMix64 generator that draws the k-means sample
 *          (uniform, without replacement, of min(n_learn, kmeans_sample)
 *          rows, Appendix A) and the k-means++ seeding draws.
 * opts     see gv_fit_opts; may be NULL.
 *
 * Steps, all in FP64: normalise the sample and run spherical k-means
 * (k-means++ seeding on the squared chord distance, Lloyd steps until no
 * assignment changes); tag every learn vector by arg-max <x, mu_c> (Eq. 9,
 * lowest c on ties); accumulate the uncentered second moments
 * K_Q = (1/m_learn) sum q q^T and K_{X_c} = sum_{x in X_c} x x^T
 * (Section 3.2); W = K_Q^(1/2) with its pseudo-inverse W+ (eigenvalues below
 * D * 2^-52 * lambda_max dropped, Section 3); for each cluster, P_c = the d
 * leading eigenvectors of W K_{X_c} W (rows, sign-fixed so that each row's
 * largest-magnitude entry is positive), A_c = P_c W+ and B_c = P_c W.
 * A cluster with fewer than d learn vectors uses the projection of the pooled
 * statistics sum_c K_{X_c}.
 *
 * Errors: GV_EINVAL (sizes), GV_ENONFINITE (NaN/Inf in the inputs),
 * GV_ENOMEM, GV_EDEVICE.  Synchronises `stream` before returning.
 */
gv_status gv_fit(const float* X_learn, int64_t n_learn, const float* Q_learn, int64_t m_learn,
                 int32_t D, int32_t d, int32_t C, uint64_t seed, const gv_fit_opts* opts,
                 void* stream, gv_model** out);

/*
 * gv_model_import -- build a model from given landmarks and projections
 * (for instance from another fit).  mu: host C x D, A and B: host C x d x D,
 * all FP64, copied.  Errors: GV_EINVAL, GV_ENONFINITE, GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_model_import(const double* mu, const double* A, const double* B,
                          int32_t C, int32_t d, int32_t D, gv_model** out);

/* Shape of a model. */
gv_status gv_model_shape(const gv_model* model, int32_t* C, int32_t* d, int32_t* D);

/* gv_model_export -- copy mu (C x D), A and B (C x d x D) to host FP64 arrays;
 * any pointer may be NULL to skip it. */
gv_status gv_model_export(const gv_model* model, double* mu, double* A, double* B);

/*
 * gv_model_stats -- fit diagnostics, host arrays, any may be NULL:
 * KQ (D x D, the mean second moment of the learn queries), KX (C x D x D,
 * per-cluster sums), lam_Q (D, eigenvalues of K_Q, decreasing), lam_c
 * (C x D, eigenvalues of W K_{X_c} W, decreasing), counts (C learn vectors
 * per cluster), fallback (C flags: pooled projection used), iters (k-means
 * centre updates).  Imported models (and loaded files without statistics)
 * return GV_EUNSUPPORTED.
 */
gv_status gv_model_stats(const gv_model* model, double* KQ, double* KX, double* lam_Q,
                         double* lam_c, int64_t* counts, uint8_t* fallback, int32_t* iters);

/*
 * gv_model_sphering -- the sphering factors of a fitted model (Section 3: W
 * with W W = K_Q, its pseudo-inverse W+) and the per-cluster projections P_c
 * with A_c = P_c W+, B_c = P_c W (Algorithm 2 through the eigendecompositions
 * of Section 3.2).  Host FP64 arrays, any may be NULL: W, Wp D x D; P C x d x D.
 * Imported models return GV_EUNSUPPORTED.
 */
gv_status gv_model_sphering(const gv_model* model, double* W, double* Wp, double* P);

/*
 * gv_model_save / gv_model_load -- the model as one file: landmarks mu, the
 * projections A_c and B_c and, for fitted models, the FP64 statistics K_Q
 * (mean) and K_{X_c} (sums), the eigenvalues, W, W+, P_c, the per-cluster
 * counts and fallback flags and the k-means step count -- everything from
 * which Section 3.2 recomputes the projections (for instance after streaming
 * updates of the statistics).  Loading restores every value bit for bit into a
 * new handle on the current device, so a search with it returns what the saved
 * model's returns; gv_model_stats and gv_model_sphering work on it when the
 * file holds statistics.  The file is little-endian binary:
 *   "GLEANVEC", u32 version (1), u32 flags (bit 0: statistics), i32 C, d, D,
 *   iters; f64 mu[C*D], A[C*d*D], B[C*d*D]; with statistics f64 KQ[D*D],
 *   KX[C*D*D], lam_Q[D], lam_c[C*D], W[D*D], W+[D*D], P[C*d*D], i64 counts[C],
 *   u8 fallback[C]; then the 64-bit FNV-1a of every preceding byte.
 * path: host NUL-terminated file name (overwritten by gv_model_save).
 * Errors: GV_ENOTFIT, GV_EINVAL (NULL path, unreadable or corrupt file: bad
 * magic, header, size or checksum), GV_EUNSUPPORTED (other file version),
 * GV_ENOMEM, GV_EDEVICE (device copies, write failure).
 */
gv_status gv_model_save(const gv_model* model, const char* path);
gv_status gv_model_load(const char* path, gv_model** out);

/*
 * gv_model_file_info -- validate a model file (magic, version, shape, size,
 * checksum) without touching the device, and return its shape (any pointer
 * may be NULL; has_stats: 1 if it holds the statistics).  Errors as
 * gv_model_load's file checks.
 */
gv_status gv_model_file_info(const char* path, int32_t* C, int32_t* d, int32_t* D, int32_t* has_stats);

void gv_model_destroy(gv_model* model);

/* ------------------------------------------------------------------ encode */

/*
 * gv_encode -- index build (Section 4, Eq. 9 and Eq. 10).
 *
 * X       device, n x D FP32 database vectors (n >= 1).
 * fmt     storage format of the reduced vectors.
 * copy_X  1: the index keeps its own copy of X (for the full-dimension
 *         rerank); 0: it borrows X, which must then outlive the index and stay
 *         unchanged; 2: it keeps no full-dimension vectors (searches then
 *         rerank from the stored vectors, gv_search_flex with
 *         GV_RERANK_STORED).
 * The reduced dimension d of the model may be anything up to D (d > 256 is
 * stored, and searched through a leading part with gv_search_flex).
 *
 * Computes tag_i = arg-max_c <x_i, mu_c> in FP64 (lowest c on ties), groups the
 * rows by tag (stable: increasing ids inside a cluster), computes
 * v_i = fl32(B_{tag_i} x_i) with FP64 accumulation, and per cluster a
 * power-of-two scale s_c mapping the cluster's largest |v| into (T/2, T]
 * (T = 448 for FP8, 65504 for FP16, 1 for BF16; s_c = 1 for FP32), then stores
 * rnd(v / s_c), rounded to nearest even with saturation.
 *
 * Errors: GV_EINVAL, GV_ENOTFIT, GV_ENONFINITE, GV_ENOMEM, GV_EDEVICE.
 * Synchronises `stream` before returning.
 */
gv_status gv_encode(const gv_model* model, const float* X, int64_t n, gv_format fmt,
                    int32_t copy_X, void* stream, gv_index** out);

/* Shape of an index: id space n (rows encoded, plus rows inserted by re-projections), clusters,
 * reduced dim, padded row length (see gv_padded_dim), format. */
gv_status gv_index_shape(const gv_index* index, int64_t* n, int32_t* C, int32_t* d,
                         int32_t* d_pad, int32_t* fmt);

/*
 * gv_index_export -- host copies of the index (any pointer may be NULL):
 * tags (n, uint8, original order, 255 for removed ids), offsets (C + 1, grouped
 * segment starts), ids (rows, int32, original id of each grouped position,
 * rows = gv_index_rows), xlow (rows x d_pad
 * elements of the storage format, raw bits, grouped order, zero padded;
 * d_pad = gv_padded_dim(d)),
 * scale (C, FP32 power-of-two s_c).
 */
gv_status gv_index_export(const gv_index* index, uint8_t* tags, int64_t* offsets, int32_t* ids,
                          void* xlow, float* scale);

void gv_index_destroy(gv_index* index);

/*
 * gv_index_reproject -- streaming update of an index without the database
 * (Section 3, streaming vector search): the stored vectors y = P_c W x of `in`
 * are carried to the refitted projections as
 *     y' = P'_c W' (P_c W)^-1 y = B'_c A_c^T y
 * (A_c, B_c of old_model, B'_c of new_model; A_c^T is the inverse of B_c when
 * d = D and K_Q has full rank), vectors inserted since are encoded as
 * y' = B'_c x, and removed ones are dropped.  Requires d = D for both models and
 * the index (flexible storage of all coordinates, Section 3.3) and identical
 * landmarks (a refit from kept landmarks, gv_fit_from_stats), so every kept
 * vector keeps its cluster.
 * keep   device uint8 per id of `in` (nonzero: kept), or NULL to keep all.
 * X_new  device n_new x D FP32 inserted vectors (ids in.n .. in.n + n_new - 1),
 *        NULL when n_new == 0.
 * fmt    storage format of the new index (per-cluster scales recomputed).
 * out    a new index over the id space [0, in.n + n_new) that keeps no
 *        full-dimension vectors (search it with gv_search_flex and
 *        GV_RERANK_STORED); removed ids have no stored vector (tag 255).
 * Each y' is fl32 of an FP64 product of the exact stored values.
 * Errors: GV_EINVAL (shapes, d < D, other landmarks, nothing left),
 * GV_ENOTFIT, GV_ENONFINITE, GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_index_reproject(const gv_model* old_model, const gv_model* new_model, const gv_index* in,
                             const uint8_t* keep, const float* X_new, int64_t n_new, gv_format fmt,
                             void* stream, gv_index** out);

/* Number of vectors an index stores (its id space minus removed ids). */
gv_status gv_index_rows(const gv_index* index, int64_t* rows);

/* ------------------------------------------------------------------ search */

/*
 * gv_search -- multi-step search (Algorithm 1) with eager views (Algorithm 4).
 *
 * Q           device, m x D FP32 queries (m >= 0; m == 0 is a no-op).
 * k, kappa    1 <= k <= kappa <= min(n, 1024); kappa above a launch shape's
 *             candidate lists (see gv_scan_plan) returns GV_EUNSUPPORTED.
 * out_ids     device, m x k int32: original row ids of the k best rerank
 *             scores, ordered by (exact score desc, id asc).
 * out_scores  device, m x k FP32 (may be NULL): fl32 of the exact <q, x>
 *             computed with FP64 accumulation.
 *
 * Stages, one launch sequence on `stream`:
 *   S1  q_c = fl32(A_c q) for every cluster (FP64 accumulation), then the
 *       per-(query, cluster) power-of-two scale t and the view
 *       q^_c = rnd(q_c / t) in the view format of the index: its storage
 *       format, FP16 for FP8 storage (t = 1 for FP32);
 *   S2  for every database vector i of cluster c:
 *       s_i = s_c * t_{q,c} * <q^_c, x^_i>, FP32 accumulation on the matrix cores;
 *   S3  the kappa best s_i per query, ordered by (s_i desc, id asc);
 *   S4  exact <q, x_i> over the kappa candidates, top k.
 * Scratch memory is taken from the stream-ordered allocator: the candidate
 * lists take at most 2 GiB, or 12 GiB for batches whose scan uses many short
 * row ranges (m >= 2048 on 10M rows: 8 GiB at m = 4096), plus the views;
 * gv_scan_plan reports the figure for a shape.
 *
 * Errors: GV_EINVAL, GV_ENOTFIT, GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_search(const gv_model* model, const gv_index* index, const float* Q, int64_t m,
                    int32_t k, int32_t kappa, int32_t* out_ids, float* out_scores, void* stream);

/*
 * gv_search_lazy -- gv_search with the lazy inner product of Algorithm 3
 * instead of the eager one (Algorithm 4): no projection pass; each work item
 * of the scan computes the views q_c = fl32(A_c q) of the cluster it visits
 * (FP64 accumulation, the same arithmetic as gv_search's projection of small
 * batches) and their FP16 view, then scores as gv_search does.  Results equal
 * gv_search's bit for bit.  Exists to measure the paper's lazy alternative:
 * the exhaustive scan visits every cluster from many work items, so the
 * projections are repeated per work item.  Supported: FP16 storage, a padded
 * reduced length of 160 (gv_padded_dim(d) == 160), 1 <= m <= 16, an index that
 * keeps X, and no qpw override.  Errors: as gv_search; GV_EUNSUPPORTED
 * otherwise.
 */
gv_status gv_search_lazy(const gv_model* model, const gv_index* index, const float* Q, int64_t m,
                         int32_t k, int32_t kappa, int32_t* out_ids, float* out_scores, void* stream);

/*
 * gv_search_noalloc -- gv_search for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, stages and results as gv_search (bit for bit),
 * but the search scratch lives in a fixed array of the library, one per device,
 * of gv_search_noalloc_capacity() bytes (64 MiB): the call makes no device
 * allocation and no allocating library call (and records no profiling events).
 * The index must keep its full-dimension vectors (copy_X 0 or 1).
 * Every call on a device uses that device's one array: calls that overlap on
 * one device (other threads, or other streams not ordered with this one) race
 * and give undefined results; order them.  A search whose scratch exceeds the
 * array (large batches: the candidate lists take m x ranges x 2048 x 8 bytes)
 * returns GV_EINVAL and names the bytes it needs.
 * Errors: as gv_search; GV_EINVAL also for a search larger than the array.
 */
gv_status gv_search_noalloc(const gv_model* model, const gv_index* index, const float* Q, int64_t m,
                            int32_t k, int32_t kappa, int32_t* out_ids, float* out_scores, void* stream);

/* Bytes of the per-device scratch array of gv_search_noalloc. */
int64_t gv_search_noalloc_capacity(void);

/*
 * gv_search_batched -- Algorithm 1 for n_coll independent collections (each
 * its own model and index, query batch and outputs), as one graph launch: every
 * collection's S1-S4 sequence is captured as a branch of one HIP graph whose
 * branches run concurrently on the device.  The graph, its workspace and the
 * argument list are kept; a later call with exactly the same arguments (handles,
 * pointers, sizes, k, kappa, stream, tuning) replays the graph without host
 * work.  Per collection the results equal gv_search's.
 * models, indexes, Q, m, out_ids, out_scores: host arrays of n_coll entries
 * (out_scores may be NULL, or hold NULL entries); m[i] == 0 skips a collection.
 * Arguments as gv_search; all indexes on the current device.
 * Collections run on four device streams (collection i on stream i % 4); the
 * kept workspace holds, per stream, the largest search scratch of its
 * collections, and stays allocated until a call with other arguments, or
 * gv_batch_release.
 * Calls that overlap (other threads) are serialised.
 * Errors: as gv_search; GV_EDEVICE if capture or instantiation fails.
 */
gv_status gv_search_batched(int32_t n_coll, const gv_model* const* models, const gv_index* const* indexes,
                            const float* const* Q, const int64_t* m, int32_t k, int32_t kappa,
                            int32_t* const* out_ids, float* const* out_scores, void* stream);

/* gv_batch_release -- free the graph and workspace kept by gv_search_batched. */
void gv_batch_release(void);

/* gv_batch_counts -- how many gv_search_batched calls since the library was
 * loaded captured a new graph and how many replayed the kept one (either
 * pointer may be NULL).  A handle enters the replay key by a generation number
 * unique to it, so a model or index destroyed and another created at the same
 * address leads to a new capture. */
void gv_batch_counts(int64_t* captures, int64_t* replays);

/*
 * gv_project -- stage S1 alone (Algorithm 4, preprocess).
 * Q device m x D FP32.  qc device m x C x d_pad FP32 (may be NULL): q_c,
 * zero padded, d_pad = gv_padded_dim(d).  t device m x C FP32: the scales.  qhat device m x C x d_pad
 * elements of the view format of `fmt` -- `fmt` itself, FP16 (2 bytes) for
 * GV_FP8_E4M3 -- (raw bits, zero padded).  Errors as gv_search.
 */
gv_status gv_project(const gv_model* model, gv_format fmt, const float* Q, int64_t m,
                     float* qc, float* t, void* qhat, void* stream);

/*
 * gv_score_topk -- stages S2 and S3 for views produced by gv_project.
 * qhat, t  device, as written by gv_project for this index's format.
 * cand_ids device m x kappa int32, cand_scores device m x kappa FP32:
 * the kappa best reduced scores per query, ordered by (score desc, id asc);
 * ids are original row ids.  1 <= kappa <= min(n, 1024).  Errors as gv_search.
 */
gv_status gv_score_topk(const gv_index* index, const void* qhat, const float* t, int64_t m,
                        int32_t kappa, int32_t* cand_ids, float* cand_scores, void* stream);

/*
 * gv_rerank -- stage S4 (Algorithm 1, postprocessing); the index must keep X.
 * Q device m x D FP32; cand_ids device m x kappa int32 (valid original ids);
 * out_ids device m x k int32, out_scores device m x k FP32 (may be NULL):
 * the k best exact <q, x> (FP64 accumulation) among the candidates, ordered by
 * (score desc, id asc).  1 <= k <= kappa <= 1024.  Errors as gv_search.
 */
gv_status gv_rerank(const gv_index* index, const float* Q, int64_t m, const int32_t* cand_ids,
                    int32_t kappa, int32_t k, int32_t* out_ids, float* out_scores, void* stream);

/* ------------------------------------------------------------------ Euclidean distance */

/* What gv_augment appends. */
enum {
  GV_AUG_DATABASE = 0,  /* -||v||^2 / 2 */
  GV_AUG_QUERY = 1      /* 1 */
};

/*
 * gv_augment -- one appended coordinate that turns Euclidean nearest
 * neighbours into maximum inner products (the paper's appendix on adapting
 * other similarities): x^ = [x, -||x||^2 / 2] for database vectors,
 * q^ = [q, 1] for queries, so <q^, x^> = -||q - x||^2 / 2 + ||q||^2 / 2.
 * Fit, encode and search then run unchanged on the D + 1 dimensional vectors.
 *
 * V    device n x D FP32.  out  device n x (D + 1) FP32 (must not alias V):
 *      row i is V's row i followed by the appended value, which for the
 *      database is the FP64 sum of the exact squares times -1/2, rounded once
 *      to FP32.
 * Errors: GV_EINVAL, GV_EDEVICE.
 */
gv_status gv_augment(const float* V, int64_t n, int32_t D, int32_t kind, float* out, void* stream);

/* ------------------------------------------------------------------ flexible d */

/* Rerank source of gv_search_flex. */
enum {
  GV_RERANK_FULL = 0,   /* exact <q, x> from the full-dimension X the index keeps */
  GV_RERANK_STORED = 1  /* <A_c q, s_c x^> over every stored coordinate */
};

/*
 * gv_search_flex -- Algorithm 1 with the reduced dimension chosen at search
 * time (Section 3.3).  The rows of each P_c are ordered by decreasing
 * eigenvalue, so the leading d_search coordinates of the stored vectors are
 * the d_search-dimensional reduction; an index encoded from a model fitted at
 * a larger d (up to D) serves every d_search <= d without re-encoding.
 *
 * d_search    1 <= d_search <= d, gv_padded_dim(d_search) <= 256.
 * rerank      GV_RERANK_FULL: exact <q, x> from the full-dimension X (the
 *             index must keep it); GV_RERANK_STORED: <A_c q, x'> with
 *             x' = s_c x^ the stored vector over all of its d coordinates and
 *             q_c = fl32(A_c q), FP64 accumulation -- with d = D this is
 *             <q, x> up to the storage rounding, and no second copy of the
 *             database is needed.
 * Other arguments and outputs as gv_search.  S1 computes q_c over all d rows;
 * the scale t and the view q^ come from its first d_search values; S2 reads
 * the leading gv_padded_dim(d_search) coordinates of every stored row.
 *
 * Errors: as gv_search; GV_EINVAL also for an out-of-range d_search, or for
 * GV_RERANK_FULL on an index that keeps no X.
 */
gv_status gv_search_flex(const gv_model* model, const gv_index* index, const float* Q, int64_t m,
                         int32_t k, int32_t kappa, int32_t d_search, int32_t rerank,
                         int32_t* out_ids, float* out_scores, void* stream);

/*
 * gv_project_flex -- stage S1 of gv_search_flex.  qc device m x C x d_pad FP32
 * (d_pad = gv_padded_dim(d); may be NULL): q_c over all d rows, zero padded.
 * t device m x C FP32: scales of the first d_search values.  qhat device
 * m x C x gv_padded_dim(d_search) elements of the view format of `fmt` (FP16
 * for GV_FP8_E4M3, else `fmt`): the views of the first
 * d_search values, zero padded.  Errors as gv_search_flex.
 */
gv_status gv_project_flex(const gv_model* model, gv_format fmt, const float* Q, int64_t m,
                          int32_t d_search, float* qc, float* t, void* qhat, void* stream);

/*
 * gv_score_topk_flex -- stages S2 and S3 on the leading d_search coordinates,
 * for views written by gv_project_flex with the same d_search.  Outputs as
 * gv_score_topk.  Errors as gv_search_flex.
 */
gv_status gv_score_topk_flex(const gv_index* index, const void* qhat, const float* t, int64_t m,
                             int32_t d_search, int32_t kappa, int32_t* cand_ids, float* cand_scores,
                             void* stream);

/*
 * gv_rerank_stored -- stage S4 from the stored vectors (Section 3.3).
 * qc device m x C x d_pad FP32 as written by gv_project_flex (or gv_project);
 * cand_ids device m x kappa int32 (original ids; negative entries are
 * skipped).  out_ids device m x k int32, out_scores device m x k FP32 (may
 * be NULL): the k best <q_c, s_c x^_i> (c the candidate's cluster, FP64
 * accumulation over all d_pad coordinates), ordered by (score desc, id asc).
 * Errors as gv_search.
 */
gv_status gv_rerank_stored(const gv_index* index, const float* qc, int64_t m, const int32_t* cand_ids,
                           int32_t kappa, int32_t k, int32_t* out_ids, float* out_scores, void* stream);

/*
 * gv_search_tuning -- override the launch shape of S2/S3 for the calling
 * thread's following searches (0 restores the automatic choice):
 * splits = row ranges per query block (1..4096), qpw = queries per wavefront
 * (32, 64 or 128), cap = key slots per (query, row range) list; a list is
 * compacted to its kappa best (ties at the kappa-th score kept) when it may
 * overflow before the next check (64..2048; a search whose launch shapes leave
 * a list no room above kappa -- see gv_scan_plan's list_limit -- fails with
 * GV_EINVAL or GV_EUNSUPPORTED).  Results
 * do not depend on these; only speed does.  Errors: GV_EINVAL.
 */
gv_status gv_search_tuning(int32_t splits, int32_t qpw, int32_t cap);

/*
 * gv_search_optimism -- the seeds of the cascade's levels after the first
 * filtering one, for the calling thread's following searches, when the level
 * before the full scan filters (three or more levels).  Algorithm 1 needs the
 * kappa best reduced scores; any score at or below a query's kappa-th best is a
 * valid threshold.  By default (rank 0) a level starts from the kappa_opt-th
 * best score of the level before, kappa_opt = f kappa + 6 sqrt(f kappa) + 6
 * with f the fraction of the level's rows the level before samples, which
 * keeps about kappa_opt / f keys instead of kappa / f.  A query whose
 * full-scan lists then hold fewer than kappa keys (its threshold was above its
 * kappa-th best) is rescanned from the exact seed, so results are exactly
 * those of the plain scan; a sample level that keeps fewer than kappa keys
 * leaves the exact seed of the level before in place.  rank > 0 takes the
 * rank-th best score instead (small ranks force rescans: for tests); rank = -1
 * starts every level from the exact kappa-th best.  Results do not depend on
 * it.  Errors: GV_EINVAL (rank < -1).
 */
gv_status gv_search_optimism(int32_t rank);

/*
 * gv_debug_fail_alloc -- for tests of the out-of-memory paths: after `after`
 * more device allocations by the library (any thread), the next one fails as if
 * the device were out of memory; the call that made it returns GV_ENOMEM and
 * releases what it had allocated.  -1 turns it off.  Allocations of the
 * caller's framework (e.g. torch tensors) are not counted.
 * Errors: GV_EINVAL (after < -1).
 */
gv_status gv_debug_fail_alloc(int32_t after);
/* the count gv_debug_fail_alloc set, less the allocations made since; -1 once
 * the failure has happened (or when off) */
int32_t gv_debug_allocs_pending(void);

/* One level of the S2/S3 launch plan (gv_scan_plan). */
typedef struct {
  int64_t stride;            /* the level scans every stride-th 32-row tile (1: the whole database) */
  int64_t rows_per_level;    /* stored rows the level visits */
  int64_t query_blocks;      /* blocks of queries_per_wave queries */
  int32_t dense;             /* 1: dense sample (every score written), 0: filtered candidate lists */
  int32_t ranges;            /* R: row ranges per query block (one candidate list each) */
  int32_t grid;              /* workgroups of 256 threads */
  int32_t queries_per_wave;  /* 32, 64 or 128 */
  int32_t shared;            /* 1: one query block on four ranges per workgroup */
  int32_t xcd_map;           /* 1: workgroups sharing rows pinned to one XCD */
  int32_t tile_ring;         /* 1: tiles shared by the workgroup through an LDS ring */
  int32_t workgroups_per_cu; /* occupancy the kernel is built for */
  int32_t check_every;       /* U: tiles between two overflow checks of a list */
  int32_t staging;           /* keys a compaction stages in the wavefront's LDS */
  int32_t list_cap;          /* key slots per (query, range) list */
  int32_t list_limit;        /* a list holding more keys is compacted to its kappa best */
} gv_scan_level;

/*
 * gv_scan_plan -- the launch plan of stages S2 and S3 for an index of n rows
 * stored as n_pad (every cluster segment padded to whole 32-row tiles, so
 * n <= n_pad <= n + 31 C, a multiple of 32), C clusters, format fmt, reduced
 * dimension d, a scan of the leading d_search coordinates (0: all of d), m
 * queries and kappa candidates, under the calling thread's gv_search_tuning.
 * Host only: computes what gv_score_topk would launch, without a device.
 * levels (host, max_levels entries, may be NULL) receives the cascade levels,
 * sparsest first; n_levels their count; list_keys the candidate-list slots of
 * the scratch (m x max ranges x list_cap); scratch_bytes the scan's scratch.
 * Errors: GV_EINVAL (sizes), GV_EUNSUPPORTED (a plan gv_score_topk would
 * refuse: too many list slots for the batch, kappa beyond a shape's lists).
 */
gv_status gv_scan_plan(int64_t n, int64_t n_pad, int32_t C, gv_format fmt, int32_t d, int32_t d_search, int64_t m,
                       int32_t kappa, gv_scan_level* levels, int32_t max_levels, int32_t* n_levels,
                       int64_t* list_keys, int64_t* scratch_bytes);

/* Result of gv_autotune. */
typedef struct {
  int32_t splits, qpw, cap;  /* the fastest launch shape (0: automatic) */
  double ms;                 /* its time per search */
  double ms_automatic;       /* the automatic shape's time per search */
  int32_t candidates;        /* shapes timed */
} gv_tune_result;

/*
 * gv_autotune -- time candidate launch shapes of stages S2/S3 (row ranges per
 * query block, queries per wavefront, list capacity; the automatic choice
 * among them) on this index with these m queries, `reps` searches each on
 * `stream`, and keep the fastest for the search's shape class -- storage
 * format, padded reduced length, batch class (1, <= 32, <= 64, <= 256, <= 1024,
 * <= 4096, more) and size class (floor(log2 stored rows)) -- in a process-wide
 * table.  Later searches of that class (gv_search, gv_search_batched, ...) use
 * the table's shape unless the thread set overrides with gv_search_tuning.
 * Results never depend on the launch shape, only speed does.  Q: device
 * m x D FP32; the index must keep X.  out (host, may be NULL) receives the
 * choice.  Synchronises `stream`.  Errors: as gv_search; GV_EUNSUPPORTED if no
 * candidate can run the search.
 */
gv_status gv_autotune(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int32_t k,
                      int32_t kappa, int32_t reps, gv_tune_result* out, void* stream);

/* The autotuner's table as a text file (one line per shape class:
 * fmt d_pad batch_class size_class splits qpw cap ms), written or merged into
 * the process's table.  Errors: GV_EINVAL (path, malformed line), GV_EDEVICE. */
gv_status gv_tuning_table_save(const char* path);
gv_status gv_tuning_table_load(const char* path);
/* The table's launch shape for a class, GV_EUNSUPPORTED if it has none. */
gv_status gv_tuning_lookup(int32_t fmt, int32_t d_pad, int64_t m, int64_t n_rows, int32_t* splits, int32_t* qpw,
                           int32_t* cap);
/* Empty the table. */
void gv_tuning_table_clear(void);

/*
 * gv_padded_dim -- the padded row length d_pad used for a reduced dimension d:
 * the smallest of 32, 64, 128, 160, 192, 256 that is >= d (gv_project and
 * gv_index_export lay rows out with it).  Returns 0 for d < 1.
 */
int32_t gv_padded_dim(int32_t d);

/*
 * gv_profile_enable / gv_profile_read -- measurement hooks for benchmarks.
 * While enabled (on != 0), every scan of the whole database (S2/S3) and every
 * final top-kappa select is bracketed by HIP events recorded on the stream it
 * runs on.  gv_profile_read waits for the recorded events, returns the summed
 * durations (milliseconds) and launch counts of the scan and of the select
 * (any pointer may be NULL), and clears the record.  Off by default; enabling
 * it costs two event records per launch.
 */
gv_status gv_profile_enable(int32_t on);
gv_status gv_profile_read(double* ms_score, int64_t* n_score, double* ms_merge, int64_t* n_merge);

/* ------------------------------------------------------------------ loss */

/*
 * gv_tags -- cluster tags of rows (the cluster-tag equation of Section 4):
 * tags[i] = arg-max_c <x_i, mu_c> in FP64, lowest c on ties.
 * X device n x D FP32 (D of the model); tags device n uint8.
 * Errors: GV_EINVAL, GV_ENOTFIT, GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_tags(const gv_model* model, const float* X, int64_t n, uint8_t* tags, void* stream);

/*
 * gv_moments -- uncentered second-moment sums (Section 3, the statistics of
 * the loss rewrite): K[c] = sum over rows v of V with tags[i] == c of v v^T,
 * FP64 accumulation of exact FP32 products.
 * V device n x D FP32; tags device n uint8 (< C), or NULL with C == 1 (every
 * row; n == 0 needs no tags); K device C x D x D FP64, overwritten.
 * Synchronises `stream`.
 * Errors: GV_EINVAL (tag >= C, bad sizes), GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_moments(const float* V, int64_t n, int32_t D, const uint8_t* tags, int32_t C, double* K,
                     void* stream);

/* ------------------------------------------------------------------ streaming */

/*
 * gv_moments_update -- streaming update of the statistics (Section 3,
 * streaming vector search): K[c] += sign * sum over rows v of V with
 * tags[i] == c of v v^T, FP64 accumulation of exact FP32 products.  sign +1
 * for inserted vectors, -1 for removed ones (their tags as when inserted, e.g.
 * from gv_tags).  Arguments otherwise as gv_moments; K is read and written.
 * Synchronises `stream`.  Errors: GV_EINVAL (tag >= C, bad sizes, sign),
 * GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_moments_update(const float* V, int64_t n, int32_t D, const uint8_t* tags, int32_t C,
                            int32_t sign, double* K, void* stream);

/*
 * gv_fit_from_stats -- the projections of a model recomputed from statistics
 * the caller keeps (Section 3, streaming vector search: the SVDs of
 * Algorithm 2 replaced by the eigendecompositions of K_Q and W K_{X_c} W).
 * mu      host C x D FP64 landmarks (kept from an earlier fit).
 * KQ      device D x D FP64: sum of q q^T over m_q learn queries.
 * KX      device C x D x D FP64: per-cluster sums of x x^T.
 * counts  host C int64: vectors behind each K_{X_c}; a cluster with fewer
 *         than d takes the projection of the pooled statistics.
 * Builds W = K^{1/2} and W+ from K_Q / m_q, P_c = top-d eigenvectors of
 * W K_{X_c} W, A_c = P_c W+, B_c = P_c W, exactly as gv_fit does after its
 * statistics; gv_model_stats then reports these statistics (K_Q as a mean).
 * Errors: GV_EINVAL, GV_ENONFINITE, GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_fit_from_stats(const double* mu, const double* KQ, double m_q, const double* KX,
                            const int64_t* counts, int32_t C, int32_t d, int32_t D, void* stream,
                            gv_model** out);

/*
 * gv_loss_grad -- the inner-product approximation loss of Problem 3 summed
 * over clusters, and its gradient, through the second-moment rewrite of
 * Section 3 (Eq. 5):
 *   L = (1/N) sum_c sum_q sum_{x in X_c} (<A_c q, B_c x> - <q, x>)^2
 *     = (1/N) sum_c <K_Q M_c K_c, M_c>_F,        M_c = A_c^T B_c - I,
 *   dL/dA_c = (2/N) B_c K_c M_c^T K_Q,   dL/dB_c = (2/N) A_c K_Q M_c K_c,
 * with K_Q = sum_q q q^T and K_c = sum_{x in X_c} x x^T (sums, e.g. from
 * gv_moments).  Evaluated in FP64 with products of at most d x D x D.
 * A, B    device C x d x D FP32 (row c*d + i is row i of A_c / B_c).
 * KQ      device D x D FP64; KX device C x D x D FP64 (symmetric).
 * n_pairs N > 0.
 * loss    device FP64 scalar; dA, dB device C x d x D FP32, either may be
 *         NULL (not computed).
 * Errors: GV_EINVAL (sizes, NULL loss/A/B/KQ/KX, N not positive and finite),
 * GV_ENOMEM, GV_EDEVICE.
 */
gv_status gv_loss_grad(int32_t C, int32_t d, int32_t D, const float* A, const float* B, const double* KQ,
                       const double* KX, double n_pairs, double* loss, float* dA, float* dB, void* stream);

/*
 * gv_host_eigh -- the host FP64 symmetric eigensolver the fit uses for the
 * eigendecompositions of Section 3.2 (Householder tridiagonalisation, then
 * implicit QR steps with Wilkinson shifts).  A: host n x n symmetric, read
 * only; lam: host n eigenvalues, decreasing; Vt: host n x n, row r is the unit
 * eigenvector of lam[r].  Runs on the CPU only.  Errors: GV_EINVAL, GV_ENOCONV.
 */
gv_status gv_host_eigh(int32_t n, const double* A, double* lam, double* Vt);

/*
 * gv_eig_step_limit -- the budget of implicit QR steps of one decomposition by
 * the host eigensolver (0, the default: 60 times the matrix order).  When a
 * decomposition needs more, gv_host_eigh, gv_fit and gv_fit_from_stats return
 * GV_ENOCONV instead of projections from an unconverged solve.  Process-wide.
 * Small budgets exist to exercise that error path.  Errors: GV_EINVAL
 * (negative budget).
 */
gv_status gv_eig_step_limit(int32_t max_steps);

#ifdef __cplusplus
}
#endif
#endif /* GLEANVEC_H */
