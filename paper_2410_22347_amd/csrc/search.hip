// Search path on gfx950: eager views (S1), grouped reduced scoring (S2) fused
// with a per-query top-kappa filter (S3), merge of the partial lists, and the
// full-dimension rerank (S4).  Algorithm 1 of the paper with the eager inner
// product of Algorithm 4 and an exhaustive main step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "search_kernels.hpp"

namespace gv {

// ============================================================================ S1
namespace {

// One wavefront per (query, cluster): amax of q_c, power-of-two scale t, the
// storage-format view rnd(q_c / t) (zero padded); also zero-pads q_c.
template <int FMT>
__global__ void k_quant_queries(float* __restrict__ qc, int64_t m, int C, int d, int dp, double T,
                                float* __restrict__ t_out, void* __restrict__ qhat) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (w >= m * C) return;
  float* v = qc + w * dp;
  float amax = 0.0f;
  for (int j = lane; j < d; j += 64) amax = fmaxf(amax, fabsf(v[j]));
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
  const float t = (FMT == GV_FP32) ? 1.0f : pow2_scale(amax, T);
  if (lane == 0) t_out[w] = t;
  for (int j = lane; j < dp; j += 64) {
    float x = (j < d) ? v[j] : 0.0f;
    if (j >= d) v[j] = 0.0f;
    double y = (double)x / (double)t;  // exact: t is a power of two
    if (FMT == GV_FP32) ((float*)qhat)[w * dp + j] = x;
    else if (FMT == GV_FP16) ((uint16_t*)qhat)[w * dp + j] = to_fp16(y);
    else if (FMT == GV_BF16) ((uint16_t*)qhat)[w * dp + j] = to_bf16(y);
    else ((uint8_t*)qhat)[w * dp + j] = to_fp8(y);
  }
}

// q_c = fl32(A_c q) for a few queries: one wavefront per row of the stacked A
// (C*d rows), the row read once and dotted with every query (FP64 accumulation).
// Used when the batch is too small to fill the GEMM tiles.
constexpr int kSmallM = 16;
__global__ __launch_bounds__(256) void k_project_small(const float* __restrict__ Q, int64_t m, int D,
                                                       const double* __restrict__ A, int64_t rows, int d, int dp,
                                                       int C, float* __restrict__ qc) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= rows) return;
  const double* a = A + j * D;
  const int64_t c = j / d, jj = j - c * d;
  for (int64_t i = 0; i < m; ++i) {
    const float* q = Q + i * D;
    double s = 0.0;
    for (int k = lane; k < D; k += 64) s += a[k] * (double)q[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) qc[(i * C + c) * dp + jj] = (float)s;
  }
}

}  // namespace

gv_status project_impl(const gv_model* model, int fmt, const float* Q, int64_t m, float* qc, float* t, void* qhat,
                       hipStream_t st) {
  const int C = model->C, d = model->d, D = model->D, dp = pad_dim(d);
  float* tmp = nullptr;
  if (!qc) {
    GV_HIP(hipMallocAsync((void**)&tmp, sizeof(float) * m * C * dp, st));
    qc = tmp;
  }
  // q_c = fl32(A_c q), FP64 accumulation; columns j of the stacked A map to (c, j % d)
  gv_status s = GV_OK;
  if (m <= kSmallM) {
    const int64_t rows = (int64_t)C * d;
    hipLaunchKernelGGL(k_project_small, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, Q, m, D, model->A, rows,
                       d, dp, C, qc);
  } else {
    GemmOperand<float> qo{Q, D, nullptr, Layout::RowMajor};
    GemmOperand<double> ao{model->A, D, nullptr, Layout::RowMajor};
    s = gemm_f64<float, double>(m, (int64_t)C * d, D, qo, ao, Epi::StoreF32Proj,
                                GemmOut{qc, (int64_t)C * dp, d, dp, nullptr}, st);
  }
  if (s == GV_OK) {
    const unsigned grid = (unsigned)((m * C + 3) / 4);
    const double T = scale_target(fmt);
    switch (fmt) {
      case GV_FP32: hipLaunchKernelGGL(k_quant_queries<GV_FP32>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, T, t, qhat); break;
      case GV_FP16: hipLaunchKernelGGL(k_quant_queries<GV_FP16>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, T, t, qhat); break;
      case GV_BF16: hipLaunchKernelGGL(k_quant_queries<GV_BF16>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, T, t, qhat); break;
      default: hipLaunchKernelGGL(k_quant_queries<GV_FP8_E4M3>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, T, t, qhat); break;
    }
  }
  if (tmp) GV_HIP(hipFreeAsync(tmp, st));
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

namespace {
using namespace scan;

// seed[q] = -inf
__global__ void k_seed_init(int64_t m, float* __restrict__ seed) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) seed[q] = -INFINITY;
}

// after the dense scan: seed = kappa-th best score of the sample (one wavefront per query)
__global__ __launch_bounds__(256) void k_dense_select(const float* __restrict__ dense, int64_t m, int64_t ns,
                                                      int kappa, float* __restrict__ seed) {
  __shared__ uint32_t hist[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  if (q >= m) return;
  const float* row = dense + q * ns;
  int valid = 0;
  for (int64_t i = lane; i < ns; i += 64) valid += row[i] != -INFINITY;
  for (int o = 32; o > 0; o >>= 1) valid += __shfl_xor(valid, o);
  float tau = -INFINITY;
  if (valid >= kappa) {
    auto load = [&](int i) { return make_key(row[i], (uint32_t)i); };
    tau = key_score(wave_kth(load, (int)ns, kappa, hist[wave]));
  }
  if (lane == 0) seed[q] = fmaxf(seed[q], tau);
}

// ---------------------------------------------------------------------------- select
// Top kappa of the R lists of one query (one workgroup per query).  The lists
// are streamed through an LDS window: each window is appended to the best
// kappa so far and cut back to kappa by a radix select.  Keys are ordered by
// (score desc, stored row asc) in the lists; the final level re-keys them by
// original id, so ties resolve by (score desc, id asc).
// FINAL: the kappa best, sorted, as (ids, scores) (-1 / NaN past the end when
// fewer exist).  Otherwise: seed[q] = max(seed[q], kappa-th best score).
constexpr int kSelWin = 4096;
constexpr int kMaxLists = 4096;

template <bool FINAL>
__global__ __launch_bounds__(256) void k_select(const uint64_t* __restrict__ buf, const int32_t* __restrict__ cnt,
                                                int R, int cap, int kappa, const int32_t* __restrict__ ids,
                                                float* __restrict__ seed, int32_t* __restrict__ out_ids,
                                                float* __restrict__ out_scores) {
  __shared__ uint64_t keys[kSelWin];
  __shared__ int32_t pre[kMaxLists + 1];
  __shared__ uint64_t stage[256];
  __shared__ int32_t wsum[4];
  __shared__ uint32_t s_kept;
  __shared__ SelectSmem sel;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = blockIdx.x;
  const int32_t* c = cnt + q * R;

  // exclusive prefix of the list lengths
  const int per = (R + 255) / 256;
  int local = 0;
  for (int j = 0; j < per; ++j) {
    const int L = tid * per + j;
    if (L < R) local += c[L];
  }
  int incl = local;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int run = incl - local;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int j = 0; j < per; ++j) {
    const int L = tid * per + j;
    if (L < R) {
      pre[L] = run;
      run += c[L];
    }
  }
  const int64_t total = (int64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
  if (tid == 0) pre[R] = (int32_t)total;
  __syncthreads();

  int kept = 0;
  for (int64_t w0 = 0; w0 < total; w0 += kSelWin - kappa) {
    const int wn = (int)std::min<int64_t>(total - w0, kSelWin - kappa);
    for (int f = tid; f < wn; f += 256) {
      const int g = (int)(w0 + f);
      int lo = 0, hi = R - 1;  // list holding flat index g: last L with pre[L] <= g
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g) lo = mid; else hi = mid - 1;
      }
      uint64_t k = buf[(q * R + lo) * (int64_t)cap + (g - pre[lo])];
      if (FINAL) {
        const uint32_t row = 0xFFFFFFFFu - (uint32_t)k;
        k = (k & 0xFFFFFFFF00000000ull) | (uint64_t)(0xFFFFFFFFu - (uint32_t)ids[row]);
      }
      keys[kept + f] = k;
    }
    __syncthreads();
    const int n = kept + wn;
    if (n > kappa) {
      const uint64_t kth = block_kth(keys, n, kappa, sel);
      if (tid == 0) s_kept = 0;
      __syncthreads();
      for (int i = tid; i < n; i += 256)
        if (keys[i] >= kth) stage[atomicAdd(&s_kept, 1u)] = keys[i];
      __syncthreads();
      for (int i = tid; i < kappa; i += 256) keys[i] = stage[i];
      __syncthreads();
      kept = kappa;
    } else {
      kept = n;
    }
  }

  if (!FINAL) {
    if (kept < kappa) return;  // fewer than kappa candidates: no bound
    // the kappa-th best is the smallest kept key
    uint64_t mn = ~0ull;
    for (int i = tid; i < kept; i += 256) mn = std::min(mn, keys[i]);
    for (int o = 32; o > 0; o >>= 1) mn = std::min(mn, (uint64_t)__shfl_xor(mn, o));
    if (lane == 0) stage[wave] = mn;
    __syncthreads();
    if (tid == 0) {
      const uint64_t m4 = std::min(std::min(stage[0], stage[1]), std::min(stage[2], stage[3]));
      seed[q] = fmaxf(seed[q], key_score(m4));
    }
    return;
  }
  // bitonic sort of 256 keys, descending (padding keys are 0)
  stage[tid] = tid < kept ? keys[tid] : 0;
  __syncthreads();
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int i = tid, j = i ^ stride;
      if (j > i) {
        const bool desc = (i & size) == 0;
        const uint64_t x = stage[i], y = stage[j];
        if (desc ? (x < y) : (x > y)) {
          stage[i] = y;
          stage[j] = x;
        }
      }
      __syncthreads();
    }
  }
  if (tid < kappa) {
    const uint64_t k = stage[tid];
    out_ids[q * kappa + tid] = (int32_t)key_id(k);
    out_scores[q * kappa + tid] = key_score(k);
  }
}

Shape choose_shape(int fmt, int dp, int64_t m, int64_t rows, int C) {
  Shape sh;
  const int qpw_override = tuned_qpw();
  if (qpw_override > 0) {
    sh.nb = std::max(1, std::min(4, qpw_override / 32));
    sh.shared = m <= sh.nb * 32;
  } else if (m <= 32) {
    sh.shared = true; sh.nb = 1;
  } else if (m <= 64) {
    sh.shared = true; sh.nb = 2;
  } else {
    sh.shared = false; sh.nb = 4;
  }
  if (sh.shared && sh.nb > 2) sh.nb = 2;
  if (!sh.shared && sh.nb < 2) sh.nb = 2;
  if (fmt == GV_FP32) sh.nb = 1;
  if (dp > 160 && sh.nb > 2) sh.nb = 2;  // keeps the query views of the longest rows in registers
  sh.nqb = (m + 32 * sh.nb - 1) / (32 * sh.nb);
  const int64_t ntiles = rows / kRows + C;
  // about 1024 wavefronts (one per SIMD) when the query blocks share a workgroup's
  // rows, 2048 (two rounds of workgroups, which evens out ranges that hold many
  // survivors) otherwise; at least 4 tiles per range
  const int64_t waves = sh.shared ? 1024 : 2048;
  int64_t R = tuned_splits() > 0 ? tuned_splits() : std::max<int64_t>(1, waves / sh.nqb);
  R = std::min<int64_t>(R, std::max<int64_t>(1, ntiles / 4));
  R = std::min<int64_t>(R, kMaxLists);
  if (sh.shared) {
    R = (R + 3) / 4 * 4;
    sh.grid = (int)(sh.nqb * (R / 4));
    sh.xcd_map = 0;
  } else {
    const int64_t qgroups = (sh.nqb + 3) / 4;
    if (qgroups > 1 && R >= 8) R = R / 8 * 8;
    sh.xcd_map = (qgroups > 1 && R % 8 == 0) ? 1 : 0;
    sh.grid = (int)(qgroups * R);
  }
  sh.R = (int)R;
  return sh;
}

template <int MODE>
gv_status dispatch_fmt(int fmt, int dp, const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  switch (fmt) {
    case GV_FP32: return dispatch_scan<GV_FP32, MODE>(dp, sh, args, st);
    case GV_FP16: return dispatch_scan<GV_FP16, MODE>(dp, sh, args, st);
    case GV_BF16: return dispatch_scan<GV_BF16, MODE>(dp, sh, args, st);
    default: return dispatch_scan<GV_FP8_E4M3, MODE>(dp, sh, args, st);
  }
}

// Sampling strides of the threshold cascade, sparsest first: the sparsest
// sample (dense scan) holds at least 8 * kappa rows; each next level is 16 times
// denser; the last entry, 1, is the full scan.  Small databases get no cascade.
std::vector<int64_t> cascade(int64_t n, int kappa) {
  std::vector<int64_t> s{1};
  int64_t top = 0;
  for (int64_t stride = 16; n / stride >= 8LL * kappa && stride <= (1LL << 24); stride *= 16) top = stride;
  for (int64_t stride = 16; stride <= top; stride *= 16) s.insert(s.begin(), stride);
  return s;
}

// freed search scratch stays in the stream-ordered pool between calls
void keep_pool(int dev) {
  static bool done[64] = {};
  if (dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

}  // namespace

// smallest list capacity the scan accepts for a given kappa: a list is checked
// for overflow every 2P + 1 tiles (P <= 6) and takes at most 32 keys per tile
int min_list_cap(int kappa) { return kappa + kRows * 13 + 1; }

gv_status score_topk_impl(const gv_index* idx, const void* qhat, const float* t, int64_t m, int kappa,
                          int32_t* cand_ids, float* cand_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  keep_pool(idx->device);
  const int fmt = idx->fmt;
  const int cap = tuned_cap() > 0 ? tuned_cap() : kCap;
  if (cap < min_list_cap(kappa) || cap > kCap) {
    set_error("candidate list capacity must lie in [kappa + 417, 2048]");
    return GV_EINVAL;
  }
  const std::vector<int64_t> levels = cascade(idx->n, kappa);
  const bool has_dense = levels.size() > 1;
  const int64_t ntiles = idx->n_pad / kRows;

  std::vector<Shape> shapes;
  int Rmax = 1;
  for (size_t li = 0; li < levels.size(); ++li) {
    const int64_t s = levels[li];
    const Shape sh = choose_shape(fmt, idx->dp, m, (ntiles + s - 1) / s * kRows, idx->C);
    if (!(has_dense && li == 0)) Rmax = std::max(Rmax, sh.R);  // the dense scan writes no lists
    shapes.push_back(sh);
  }
  const int64_t ns = has_dense ? ((ntiles + levels[0] - 1) / levels[0]) * kRows : 0;

  uint64_t* buf = nullptr;
  int32_t* cnt = nullptr;
  float* seed = nullptr;
  float* dense = nullptr;
  gv_status s = GV_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (s == GV_OK && hipMallocAsync(p, std::max<size_t>(bytes, 8), st) != hipSuccess) {
      set_error("search scratch allocation failed");
      s = GV_ENOMEM;
    }
  };
  alloc((void**)&buf, sizeof(uint64_t) * m * Rmax * cap);
  alloc((void**)&cnt, sizeof(int32_t) * m * Rmax);
  if (has_dense) {
    alloc((void**)&seed, sizeof(float) * m);
    alloc((void**)&dense, sizeof(float) * m * ns);
  }

  ScoreArgs args{};
  args.xlow = (const uint8_t*)idx->xlow;
  args.ids = idx->ids;
  args.scale = idx->scale;
  args.offsets = idx->offsets;
  args.seg_end = idx->seg_end;
  args.qhat = (const uint8_t*)qhat;
  args.qscale = t;
  args.buf = buf;
  args.cnt_out = cnt;
  args.dense = dense;
  args.m = m;
  args.n_pad = idx->n_pad;
  args.C = idx->C;
  args.dp = idx->dp;
  args.kappa = kappa;
  args.cap = cap;

  if (s == GV_OK && has_dense)
    hipLaunchKernelGGL(k_seed_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, seed);
  for (size_t li = 0; li < levels.size() && s == GV_OK; ++li) {
    const Shape& sh = shapes[li];
    const bool last = li + 1 == levels.size();
    args.seed = li == 0 ? nullptr : seed;
    args.R = sh.R;
    args.nqb = (int)sh.nqb;
    args.stride = (int)levels[li];
    args.xcd_map = sh.xcd_map;
    if (has_dense && li == 0) {
      s = dispatch_fmt<kDense>(fmt, idx->dp, sh, args, st);
      if (s == GV_OK)
        hipLaunchKernelGGL(k_dense_select, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, dense, m, ns, kappa, seed);
      continue;
    }
    if (sh.R > Rmax) {  // scratch must cover every list the launch writes
      set_error("internal: candidate scratch smaller than the launch");
      s = GV_EDEVICE;
      break;
    }
    if (last) profile_mark(st, 0, true);
    s = dispatch_fmt<kFilter>(fmt, idx->dp, sh, args, st);
    if (last) profile_mark(st, 0, false);
    if (s != GV_OK) break;
    if (last) {
      profile_mark(st, 1, true);
      hipLaunchKernelGGL(k_select<true>, dim3((unsigned)m), dim3(256), 0, st, buf, cnt, sh.R, cap, kappa, idx->ids,
                         seed, cand_ids, cand_scores);
      profile_mark(st, 1, false);
    } else {
      hipLaunchKernelGGL(k_select<false>, dim3((unsigned)m), dim3(256), 0, st, buf, cnt, sh.R, cap, kappa, idx->ids,
                         seed, (int32_t*)nullptr, (float*)nullptr);
    }
  }
  for (void* p : {(void*)buf, (void*)cnt, (void*)seed, (void*)dense})
    if (p) (void)hipFreeAsync(p, st);
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

// ============================================================================ S4
namespace {

// One workgroup per query, sixteen wavefronts; each wavefront scores four
// candidate rows at a time so their loads are in flight together.
constexpr int kRerankThreads = 1024;

__global__ __launch_bounds__(kRerankThreads) void k_rerank(const float* __restrict__ X, int64_t n, int D,
                                                           const float* __restrict__ Q,
                                                           const int32_t* __restrict__ cand, int kappa, int k,
                                                           int32_t* __restrict__ out_ids,
                                                           float* __restrict__ out_scores) {
  __shared__ double s_score[256];
  __shared__ int32_t s_id[256];
  constexpr int W = kRerankThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = blockIdx.x;
  const float* qv = Q + q * D;
  if (tid < 256) {
    s_score[tid] = -INFINITY;
    s_id[tid] = 0x7fffffff;
  }
  __syncthreads();
  // exact <q, x> with FP64 accumulation of exact FP32 x FP32 products
  for (int c0 = wave * 4; c0 < kappa; c0 += W * 4) {
    int32_t id[4];
    bool ok[4];
    const float* x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      id[u] = (c0 + u < kappa) ? cand[q * kappa + c0 + u] : -1;
      ok[u] = id[u] >= 0 && id[u] < n;  // a missing candidate (non-finite query scores) is skipped
      x[u] = X + (ok[u] ? (int64_t)id[u] : 0) * D;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < D; j += 64) {
      const double qj = (double)qv[j];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += (double)x[u][j] * qj;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double v = acc[u];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0 && ok[u]) {
        s_score[c0 + u] = v;
        s_id[c0 + u] = id[u];
      }
    }
  }
  __syncthreads();
  // bitonic sort of 256 (score, id) pairs: score desc, then id asc
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (tid < 256) {
        const int i = tid, j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const double xs = s_score[i], ys = s_score[j];
          const int32_t xi = s_id[i], yi = s_id[j];
          const bool x_better = (xs > ys) || (xs == ys && xi < yi);
          if (desc ? !x_better : x_better) {
            s_score[i] = ys;
            s_score[j] = xs;
            s_id[i] = yi;
            s_id[j] = xi;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < k; i += kRerankThreads) {
    out_ids[q * k + i] = s_id[i];
    if (out_scores) out_scores[q * k + i] = (float)s_score[i];
  }
}

}  // namespace

gv_status rerank_impl(const gv_index* idx, const float* Q, int64_t m, const int32_t* cand, int kappa, int k,
                      int32_t* out_ids, float* out_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  hipLaunchKernelGGL(k_rerank, dim3((unsigned)m), dim3(kRerankThreads), 0, st, idx->X, idx->n, idx->D, Q, cand, kappa, k, out_ids,
                     out_scores);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace gv
