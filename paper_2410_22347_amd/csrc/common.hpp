// Shared declarations of the gfx950 GleanVec library: handles, error plumbing,
// storage-format conversion and the 64-bit ordering key of the top-k stages.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gleanvec.h"

namespace gv {

constexpr int kWave = 64;
// largest kappa (candidates per query) of the select and rerank stages
constexpr int kMaxKappa = 1024;

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_error();

#define GV_HIP(...)                                                        \
  do {                                                                     \
    hipError_t _e = (__VA_ARGS__);                                         \
    if (_e != hipSuccess) {                                                \
      ::gv::set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(_e)); \
      return _e == hipErrorOutOfMemory ? GV_ENOMEM : GV_EDEVICE;           \
    }                                                                      \
  } while (0)

// Every device allocation of the library goes through dev_malloc /
// dev_malloc_async, so that a test can make one chosen allocation fail as if
// the device were out of memory (gv_debug_fail_alloc).
bool take_forced_alloc_failure();
template <typename T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
  if (take_forced_alloc_failure()) return hipErrorOutOfMemory;
  return hipMalloc((void**)p, bytes);
}
template <typename T>
inline hipError_t dev_malloc_async(T** p, size_t bytes, hipStream_t st) {
  if (take_forced_alloc_failure()) return hipErrorOutOfMemory;
  return hipMallocAsync((void**)p, bytes, st);
}
// A stream-ordered temporary, freed on its stream when the guard leaves scope
// (error returns included); release() hands it to the caller instead.
template <typename T>
struct TempBuf {
  T* p = nullptr;
  hipStream_t st;
  explicit TempBuf(hipStream_t s) : st(s) {}
  TempBuf(const TempBuf&) = delete;
  TempBuf& operator=(const TempBuf&) = delete;
  hipError_t alloc(size_t bytes) { return dev_malloc_async(&p, bytes > 0 ? bytes : 1, st); }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
  ~TempBuf() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

#define GV_TRY(...)                     \
  do {                                  \
    gv_status _s = (__VA_ARGS__);       \
    if (_s != GV_OK) return _s;         \
  } while (0)

#define GV_REQUIRE(cond, msg)           \
  do {                                  \
    if (!(cond)) {                      \
      ::gv::set_error(msg);             \
      return GV_EINVAL;                 \
    }                                   \
  } while (0)

// ---------------------------------------------------------------- formats
inline int fmt_bytes(int f) { return f == GV_FP32 ? 4 : (f == GV_FP8_E4M3 ? 1 : 2); }
// Format of the query views that meet stored vectors of format f: the storage
// format, except FP8 storage, which is scored against FP16 views (the matrix
// core takes E4M3 widened exactly to FP16; FP16 x E4M3 products are exact).
inline int view_fmt(int f) { return f == GV_FP8_E4M3 ? GV_FP16 : f; }

// Matrix-core operand tiling of the stored reduced vectors.  Rows are grouped
// by cluster, each cluster's segment padded to a multiple of 32 rows.  A tile
// is 32 consecutive rows; within it, k-step s (KM reduced dimensions) forms a
// block of 64 lanes x EPL elements where lane l holds row l % 32, dimensions
// s*KM + (l / 32)*EPL ... + EPL - 1.  A wavefront thus loads the A operand of
// one k-step as one contiguous block.  FP32: KM = 2, EPL = 1; FP16, BF16 and
// FP8: KM = 16, EPL = 8.
inline int fmt_km(int f) { return f == GV_FP32 ? 2 : 16; }
inline int fmt_epl(int f) { return f == GV_FP32 ? 1 : 8; }
constexpr int kTileRows = 32;
__host__ __device__ inline int64_t tiled_offset(int64_t p, int j, int dp, int km, int epl) {
  const int64_t t = p / kTileRows;
  const int i = (int)(p - t * kTileRows);
  const int s = j / km, w = j - s * km;
  const int half = w / epl, e = w - half * epl;
  const int lane = i + kTileRows * half;
  return (t * (dp / km) + s) * (int64_t)(64 * epl) + (int64_t)lane * epl + e;  // in elements
}
// Reduced rows (and query views) are zero-padded to one of a few lengths so
// the scoring kernel runs a fully unrolled, branch-free matrix-core chain.
inline int pad_dim(int d) {
  const int sizes[] = {32, 64, 128, 160, 192, 256};
  for (int s : sizes)
    if (d <= s) return s;
  return (d + 15) / 16 * 16;  // beyond 256: stored, scanned through a leading part of at most 256
}

// Scale targets: the block's largest magnitude is mapped into (T/2, T].
inline double scale_target(int f) {
  switch (f) {
    case GV_FP16: return 65504.0;
    case GV_BF16: return 1.0;
    case GV_FP8_E4M3: return 448.0;
    default: return 0.0;  // FP32: no scaling
  }
}

// Power-of-two s with amax/s in (T/2, T] (1 for amax == 0 or T == 0), found by
// exact comparisons against T * 2^e.
__host__ __device__ inline float pow2_scale(float amax, double T) {
  if (!(amax > 0.0f) || T == 0.0) return 1.0f;
  double a = (double)amax;
  int e = 0;
  // coarse start from the binary exponents, then exact correction
  int ea = 0, et = 0;
  (void)frexp(a, &ea);
  (void)frexp(T, &et);
  e = ea - et;
  while (a > ldexp(T, e)) ++e;
  while (a <= ldexp(T, e - 1)) --e;
  return (float)ldexp(1.0, e);
}

// Round a float64 value to the nearest value of a small binary format
// (E exponent bits, M fraction bits, given bias), ties to even, saturating at
// max_code; returns the bit pattern.  The value is scaled by an exact power of
// two so rint() (round-half-even) gives the correctly rounded significand.
template <int E, int M>
__host__ __device__ inline uint32_t round_bits(double y, int bias, double vmax, uint32_t max_code) {
  uint32_t sign = signbit(y) ? 1u : 0u;
  double a = fabs(y);
  uint32_t code;
  if (a == 0.0) {
    code = 0;
  } else {
    const int emin = 1 - bias;
    int e = ilogb(a);
    if (e < emin) e = emin;
    double r = rint(ldexp(a, M - e));          // significand in units of 2^(e-M)
    if (r >= ldexp(1.0, M + 1)) {              // carried into the next binade
      r = ldexp(1.0, M);
      e += 1;
    }
    if (ldexp(r, e - M) > vmax) {
      code = max_code;
    } else if (r < ldexp(1.0, M)) {            // subnormal (only possible at e == emin)
      code = (uint32_t)r;
    } else {
      code = ((uint32_t)(e + bias) << M) | ((uint32_t)r - (1u << M));
    }
  }
  return (sign << (E + M)) | code;
}

__host__ __device__ inline uint16_t to_fp16(double y) {
  return (uint16_t)round_bits<5, 10>(y, 15, 65504.0, 0x7BFFu);
}
__host__ __device__ inline uint16_t to_bf16(double y) {
  return (uint16_t)round_bits<8, 7>(y, 127, 3.3895313892515355e38, 0x7F7Fu);
}
__host__ __device__ inline uint8_t to_fp8(double y) {
  return (uint8_t)round_bits<4, 3>(y, 7, 448.0, 0x7Eu);
}

// Exact values of the stored bit patterns (IEEE binary16, bfloat16, OCP E4M3).
__host__ __device__ inline double from_fp16(uint16_t h) {
  const int e = (h >> 10) & 31, f = h & 1023;
  const double v = e == 0 ? ldexp((double)f, -24) : ldexp((double)(1024 + f), e - 25);
  return (h & 0x8000u) ? -v : v;
}
__host__ __device__ inline double from_bf16(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}
__host__ __device__ inline double from_fp8(uint8_t c) {
  const int e = (c >> 3) & 15, f = c & 7;
  const double v = e == 0 ? ldexp((double)f, -9) : ldexp((double)(8 + f), e - 10);
  return (c & 0x80u) ? -v : v;
}

// ---------------------------------------------------------------- ordering key
// 64-bit key ordering candidates by (score desc, id asc): larger key = better.
__host__ __device__ inline uint32_t order_f32(float s) {
  s = s + 0.0f;  // -0 -> +0
  uint32_t u;
  memcpy(&u, &s, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float unorder_f32(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  float s;
  memcpy(&s, &u, 4);
  return s;
}
__host__ __device__ inline uint64_t make_key(float s, uint32_t id) {
  return ((uint64_t)order_f32(s) << 32) | (uint64_t)(0xFFFFFFFFu - id);
}
__host__ __device__ inline float key_score(uint64_t k) { return unorder_f32((uint32_t)(k >> 32)); }
__host__ __device__ inline uint32_t key_id(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFu); }

}  // namespace gv

// ---------------------------------------------------------------- handles
struct gv_model {
  uint64_t magic;
  uint64_t gen;  // unique per handle in the process (never reused, unlike its address)
  int C, d, D;
  int device;
  double* mu;  // device C x D
  double* A;   // device C*d x D (A_c stacked)
  double* B;   // device C*d x D
  bool fitted;
  std::vector<double> KQ, KX, lamQ, lamc;
  std::vector<double> W, Wp, P;  // host D x D, D x D, C x d x D (fitted models)
  std::vector<int64_t> counts;
  std::vector<uint8_t> fallback;
  int iters;
};

struct gv_index {
  uint64_t magic;
  uint64_t gen;  // unique per handle in the process (never reused, unlike its address)
  int C, d, dp, D, fmt;
  int64_t n;       // id space: original ids lie in [0, n) (every one stored, unless removed by a re-projection)
  int64_t n_rows;  // stored vectors (n minus removed ids)
  int64_t n_pad;   // stored rows: every cluster segment padded to a multiple of 32
  int device;
  uint8_t* tags;     // device n, cluster of each original id (255: removed)
  int64_t* offsets;  // device C+1, padded segment starts (multiples of 32)
  int64_t* seg_end;  // device C, first padding row of each segment (offsets[c] + rows of c)
  int32_t* ids;      // device n_pad, original id of each stored row, -1 for padding
  int32_t* pos;      // device n, stored row of each original id (-1: removed)
  void* xlow;        // device n_pad x dp elements of fmt, matrix-core tiled
  float* scale;      // device C
  const float* X;    // device n x D (owned if own_X), NULL when the index keeps none
  bool own_X;
  std::vector<int64_t> h_offsets;  // padded segment starts
  std::vector<int64_t> h_counts;   // rows per cluster
};

constexpr uint64_t kModelMagic = 0x474C45414E4D4F44ull;  // "GLEANMOD"
constexpr uint64_t kIndexMagic = 0x474C45414E494458ull;  // "GLEANIDX"

namespace gv {
// next handle generation (1, 2, ...): keys of kept state name handles by it
uint64_t next_handle_gen();
// a model handle with device storage for mu, A, B (shape C, d, D); fitted = false
gv_status alloc_model(int C, int d, int D, gv_model** out);
bool valid_model(const gv_model* m);
// internal entry points shared between translation units
gv_status fit_impl(const float* X, int64_t n, const float* Q, int64_t m, int D, int d, int C,
                   uint64_t seed, const gv_fit_opts* opts, hipStream_t st, gv_model* model);
gv_status encode_impl(const gv_model* model, const float* X, int64_t n, int fmt, hipStream_t st,
                      gv_index* index);
// encode steps shared with the re-projection of stored vectors: grouping of the
// rows of index->tags (tags >= C absent) and the scaled storage of grouped rows
gv_status group_rows(int64_t n, int C, int dp, int fmt, hipStream_t st, gv_index* idx, int64_t** ids64_out);
gv_status quantize_rows(const float* v, int d, int fmt, hipStream_t st, gv_index* idx);
gv_status reproject_impl(const gv_model* m0, const gv_model* m1, const gv_index* in, const uint8_t* keep,
                         const float* X_new, int64_t n_new, int fmt, hipStream_t st, gv_index* out);
gv_status sphere_project(gv_model* model, const double* KX_dev, const std::vector<int64_t>& counts,
                         const double* mu_dev, hipStream_t st);
gv_status fit_from_stats_impl(const double* mu, const double* KQ, double m_q, const double* KX,
                              const int64_t* counts, hipStream_t st, gv_model* model);
// d_search (0: all of the model's d) is the number of leading coordinates the
// views and the scan use (Section 3.3); q_c always holds all d of them.
// scratch (may be null): device memory the call may overwrite, for the partial
// products of a K-split GEMM (proj_split_bytes; allocated when missing or short)
gv_status project_impl(const gv_model* model, int fmt, const float* Q, int64_t m, float* qc,
                       float* t, void* qhat, hipStream_t st, int d_search = 0, void* scratch = nullptr,
                       size_t scratch_bytes = 0);
int proj_splits(int64_t m, int64_t rows, int K);
size_t proj_split_bytes(int64_t m, int64_t rows, int K);
gv_status scan_plan_describe(int64_t n, int64_t n_pad, int C, int fmt, int d, int d_search, int64_t m, int kappa,
                             gv_scan_level* levels, int max_levels, int* n_levels, int64_t* list_keys,
                             int64_t* scratch_bytes);
gv_status score_topk_impl(const gv_index* index, const void* qhat, const float* t, int64_t m,
                          int kappa, int32_t* cand_ids, float* cand_scores, hipStream_t st, int d_search = 0);
void keep_pool(int device);
// one search's scratch, carved from a single workspace (byte offsets)
// bytes of candidate lists an automatic scan plan may take: any shape
// (kListBudget), and the many-range shape of a large single search
// (kListBudgetLarge: more, shorter row ranges keep the workgroups that share a
// range in step, so its tiles stay in L2); the searches of a batched launch
// hold their lists at the same time and keep to kListBudget
constexpr uint64_t kListBudget = 2ull << 30;
constexpr uint64_t kListBudgetLarge = 12ull << 30;
struct SearchPlan {
  size_t off_t = 0, off_qc = 0, off_qhat = 0, off_cand = 0, off_csc = 0, off_scan = 0, bytes = 0;
  uint64_t list_budget = kListBudgetLarge;  // for the many-range shape (search_run re-plans with it)
  size_t scan_bytes = 0;  // scratch of S2/S3 within the workspace (search_run re-plans and checks it)
  size_t region_bytes = 0;  // bytes at off_scan: S2/S3's scratch, earlier S1's partial products, later S4's scores
  int d_search = 0;     // leading coordinates scanned
  bool stored = false;  // rerank from the stored vectors instead of the full-dimension X
};
gv_status search_plan(const gv_model* model, const gv_index* index, int64_t m, int kappa, SearchPlan* plan,
                      int d_search = 0, bool stored = false, uint64_t list_budget = kListBudgetLarge);
gv_status search_run(const gv_model* model, const gv_index* index, const float* Q, int64_t m, int k, int kappa,
                     int32_t* out_ids, float* out_scores, const SearchPlan& plan, void* workspace, hipStream_t st);
// one search of a batched launch sequence, with its own workspace
struct BatchEntry {
  const gv_model* model;
  const gv_index* idx;
  const float* Q;
  int64_t m;
  int32_t* out_ids;
  float* out_scores;
  SearchPlan plan;
  uint8_t* ws;
};
gv_status batched_run(std::vector<BatchEntry>& entries, int k, int kappa, hipStream_t org, hipStream_t* side,
                      int nside, hipEvent_t fork, hipEvent_t* join, uint8_t* qmem, size_t qbytes, int n_cu,
                      std::vector<uint8_t>* upload);
size_t batched_queue_bytes(int n_entries);
gv_status search_lazy_impl(const gv_model* model, const gv_index* idx, const float* Q, int64_t m, int k, int kappa,
                           int32_t* out_ids, float* out_scores, hipStream_t st);
// S4; scratch (may be null): device memory the call may overwrite (dead
// candidate lists), which lets small batches spread over more workgroups
gv_status rerank_impl(const gv_index* index, const float* Q, int64_t m, const int32_t* cand,
                      int kappa, int k, int32_t* out_ids, float* out_scores, hipStream_t st,
                      void* scratch = nullptr, size_t scratch_bytes = 0);
gv_status rerank_stored_impl(const gv_index* index, const float* qc, int64_t m, const int32_t* cand,
                             int kappa, int k, int32_t* out_ids, float* out_scores, hipStream_t st);
gv_status check_finite_f32(const float* p, int64_t count, hipStream_t st, bool* finite);
gv_status augment_impl(const float* V, int64_t n, int D, int database, float* out, hipStream_t st);
gv_status tags_impl(const gv_model* model, const float* X, int64_t n, uint8_t* tags, hipStream_t st);
gv_status moments_impl(const float* V, int64_t n, int D, const uint8_t* tags, int C, double* K, hipStream_t st,
                       int sign = 0);
gv_status loss_grad_impl(int C, int d, int D, const float* A, const float* B, const double* KQ, const double* KX,
                         double n_pairs, double* loss, float* dA, float* dB, hipStream_t st);

// FP64 matrix-core GEMM: C(i, j) = sum_k a(i, k) b(j, k) with operand layouts
// described by GemmOperand; epilogue selects how C is stored.
enum class Layout { RowMajor, KMajor };
template <typename T>
struct GemmOperand {
  const T* p;
  int64_t ld;
  const int64_t* gather;  // optional: RowMajor -> row index of i; KMajor -> row index of k
  Layout layout;
  int64_t bstride = 0;    // batched products: elements between consecutive operands
};
enum class Epi { StoreF64, AddF64, StoreF32Proj, StoreF32 };
struct GemmOut {
  void* p;
  int64_t ldc;
  int cd;     // StoreF32Proj: columns per cluster (d)
  int cdp;    // StoreF32Proj: padded columns per cluster
  const int64_t* row_map;  // StoreF32: output row of i (optional)
  int64_t bstride = 0;     // batched products: elements between consecutive outputs
  double alpha = 1.0;      // every epilogue stores alpha * C
};
// batch >= 1 independent products (blockIdx.z), operands and outputs offset by
// their bstride
template <typename TA, typename TB>
gv_status gemm_f64(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a, GemmOperand<TB> b, Epi epi,
                   GemmOut out, hipStream_t st, int batch = 1);

// host symmetric eigensolver (Householder tridiagonalisation + implicit QL/QR)
// A: n x n symmetric (row-major, overwritten); lam: n eigenvalues decreasing;
// Vt: n x n, row r = unit eigenvector of lam[r].  Returns false if the QR steps
// did not converge within the step budget (set_eig_step_limit).
bool eigh_desc(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Vt);
void set_eig_step_limit(long max_steps);

int tuned_splits();
int tuned_qpw();
int tuned_cap();
int tuned_optimism();  // the optimistic seed's rank override (gv_search_optimism)
// Launch overrides of S2/S3 (0: automatic).  The calling thread's overrides
// (gv_search_tuning) come first; else the autotuner's table entry for the
// search's shape class (format, padded length, batch class, size class).
struct Tuning {
  int splits = 0, qpw = 0, cap = 0;
};
Tuning effective_tuning(int fmt, int dp, int64_t m, int64_t n_rows);
bool tuning_table_lookup(int fmt, int dp, int64_t m, int64_t n_rows, Tuning* t);
void tuning_table_store(int fmt, int dp, int64_t m, int64_t n_rows, const Tuning& t, double ms);
uint64_t tuning_table_version();
// the calling thread's launch overrides (as gv_search_tuning, unchecked)
void set_tuning(int splits, int qpw, int cap);
// smallest candidate-list capacity the scan accepts for kappa
int min_list_cap(int kappa);

// benchmark hooks: events around scoring (kind 0) and merge (kind 1) launches
// (off while a batched search is being captured into a graph)
bool profiling();
void profile_mark(hipStream_t st, int kind, bool begin);
// no profiling events (which create HIP events) on this thread while on
void suppress_profile_events(bool on);
// argument rules shared by the search entry points
gv_status check_search_args(const gv_index* idx, int64_t m, int32_t k, int32_t kappa);
}  // namespace gv
