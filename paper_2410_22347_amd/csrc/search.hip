// Search path on gfx950: eager views (S1), grouped reduced scoring (S2) fused
// with a per-query top-kappa filter (S3), merge of the partial lists, and the
// full-dimension rerank (S4).  Algorithm 1 of the paper with the eager inner
// product of Algorithm 4 and an exhaustive main step.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <vector>

#include "search_kernels.hpp"

namespace gv {

// ============================================================================ S1
namespace {

// One wavefront per (query, cluster): zero-pads q_c (row pitch dq) past its d
// values; the power-of-two scale t of its first ds values and the view
// rnd(q_c / t) of them in view format FMT (row pitch dpo, zero padded).
template <int FMT>
__global__ void k_quant_queries(float* __restrict__ qc, int64_t m, int C, int d, int dq, int ds, int dpo, double T,
                                float* __restrict__ t_out, void* __restrict__ qhat) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (w >= m * C) return;
  float* v = qc + w * dq;
  for (int j = d + lane; j < dq; j += 64) v[j] = 0.0f;
  float amax = 0.0f;
  for (int j = lane; j < ds; j += 64) amax = fmaxf(amax, fabsf(v[j]));
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
  const float t = (FMT == GV_FP32) ? 1.0f : pow2_scale(amax, T);
  if (lane == 0) t_out[w] = t;
  for (int j = lane; j < dpo; j += 64) {
    const float x = (j < ds) ? v[j] : 0.0f;
    const double y = (double)x / (double)t;  // exact: t is a power of two
    if (FMT == GV_FP32) ((float*)qhat)[w * dpo + j] = x;
    else if (FMT == GV_FP16) ((uint16_t*)qhat)[w * dpo + j] = to_fp16(y);
    else ((uint16_t*)qhat)[w * dpo + j] = to_bf16(y);
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

// S1 for batches that give the tiled GEMM few output tiles: the K loop of each
// tile is a chain of memory latencies, so K is cut into `ks` slices computed as
// independent products (FP64 partial tiles in scratch), then summed here in
// slice order and rounded once to FP32.
__global__ void k_proj_reduce(const double* __restrict__ part, int ks, int64_t m, int64_t rows, int d, int dp,
                              int C, float* __restrict__ qc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * rows) return;
  const int64_t i = e / rows, j = e - i * rows;
  double v = part[e];
  for (int z = 1; z < ks; ++z) v += part[(int64_t)z * m * rows + e];
  const int64_t c = j / d, jj = j - c * d;
  qc[(i * C + c) * dp + jj] = (float)v;
}

}  // namespace

// K slices of S1's tiled GEMM for m queries and `rows` stacked rows of A
// (length K): doubled while the output tiles (64 x 64) number fewer than 512
// and K splits evenly; decided by the shape alone, so every caller of one shape
// computes the same sums
int proj_splits(int64_t m, int64_t rows, int K) {
  if (m <= kSmallM) return 1;
  const int64_t tiles = ((m + 63) / 64) * ((rows + 63) / 64);
  int ks = 1;
  while (ks < 16 && tiles * ks < 512 && K % (2 * ks) == 0 && K / (2 * ks) >= 32) ks *= 2;
  return ks;
}

size_t proj_split_bytes(int64_t m, int64_t rows, int K) {
  const int ks = proj_splits(m, rows, K);
  return ks > 1 ? sizeof(double) * (size_t)ks * (size_t)m * (size_t)rows : 0;
}

gv_status project_impl(const gv_model* model, int fmt, const float* Q, int64_t m, float* qc, float* t, void* qhat,
                       hipStream_t st, int d_search, void* scratch, size_t scratch_bytes) {
  const int C = model->C, d = model->d, D = model->D, dp = pad_dim(d);
  const int ds = d_search > 0 ? d_search : d, dpo = pad_dim(ds);
  TempBuf<float> tmp(st);
  if (!qc) {
    GV_HIP(tmp.alloc(sizeof(float) * m * C * dp));
    qc = tmp.p;
  }
  // q_c = fl32(A_c q), FP64 accumulation; columns j of the stacked A map to (c, j % d)
  gv_status s = GV_OK;
  if (m <= kSmallM) {
    const int64_t rows = (int64_t)C * d;
    hipLaunchKernelGGL(k_project_small, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, Q, m, D, model->A, rows,
                       d, dp, C, qc);
  } else {
    const int64_t rows = (int64_t)C * d;
    const int ks = proj_splits(m, rows, D);
    GemmOperand<float> qo{Q, D, nullptr, Layout::RowMajor};
    GemmOperand<double> ao{model->A, D, nullptr, Layout::RowMajor};
    if (ks == 1) {
      s = gemm_f64<float, double>(m, rows, D, qo, ao, Epi::StoreF32Proj, GemmOut{qc, (int64_t)C * dp, d, dp, nullptr},
                                  st);
    } else {
      const size_t need = proj_split_bytes(m, rows, D);
      TempBuf<double> pbuf(st);
      double* part = (double*)scratch;
      if (!part || scratch_bytes < need) {
        GV_HIP(pbuf.alloc(need));
        part = pbuf.p;
      }
      const int kc = D / ks;
      qo.bstride = kc;
      ao.bstride = kc;
      GemmOut po{part, rows, 0, 0, nullptr};
      po.bstride = m * rows;
      s = gemm_f64<float, double>(m, rows, kc, qo, ao, Epi::StoreF64, po, st, ks);
      if (s == GV_OK)
        hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)((m * rows + 255) / 256)), dim3(256), 0, st, part, ks, m,
                           rows, d, dp, C, qc);
    }
  }
  if (s == GV_OK) {
    const unsigned grid = (unsigned)((m * C + 3) / 4);
    const int vf = view_fmt(fmt);  // FP8 storage meets FP16 views
    const double T = scale_target(vf);
    switch (vf) {
      case GV_FP32: hipLaunchKernelGGL(k_quant_queries<GV_FP32>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, ds, dpo, T, t, qhat); break;
      case GV_FP16: hipLaunchKernelGGL(k_quant_queries<GV_FP16>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, ds, dpo, T, t, qhat); break;
      default: hipLaunchKernelGGL(k_quant_queries<GV_BF16>, dim3(grid), dim3(256), 0, st, qc, m, C, d, dp, ds, dpo, T, t, qhat); break;
    }
  }
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

namespace {
using namespace scan;

// n counters to zero (a kernel rather than a memset node inside captured graphs)
__global__ void k_zero_ints(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// After an optimistic full scan (see run_scan): a query whose lists hold fewer
// than kappa keys may have missed some of its kappa best (its seed lay above its
// kappa-th best score), so its lists are emptied and it is rescanned from the
// exact seed; every other query gets +inf, which the repair pass leaves alone.
// One wavefront per query.
__global__ __launch_bounds__(256) void k_repair_prep(int32_t* __restrict__ cnt, int R, int64_t m, int kappa,
                                                     const float* __restrict__ seed,
                                                     const float* __restrict__ seed_opt, float* __restrict__ rescan) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= m) return;
  int32_t* c = cnt + q * R;
  long long total = 0;
  for (int r = lane; r < R; r += 64) total += c[r];
  for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
  const bool redo = total < kappa && seed_opt[q] > seed[q];
  if (redo)
    for (int r = lane; r < R; r += 64) c[r] = 0;
  if (lane == 0) rescan[q] = redo ? seed[q] : INFINITY;
}

// after the dense scan: seed = a lower bound of the kappa-th best score of the
// sample.  Any such bound is a valid seed (at least kappa rows of the next level
// reach it); this one is the smallest score whose order key shares the top 22
// bits of the kappa-th best's key (within 2^-13 of it, relatively), found from
// two 11-bit histograms: two passes over the row instead of the four or more of
// an exact radix select.  The optimistic seed's rank is resolved from the same
// two passes (one first-pass histogram, a second-pass histogram per rank).
constexpr int kBoundBins = 2048;
constexpr int kDenseThreads = 256;

// the bin of h (kBoundBins counts, higher bins = larger keys) holding the
// need-th largest key, and that key's rank within the bin; called by every
// thread of a kDenseThreads workgroup, which returns the same result to all
// (-1 when the bins hold fewer than need keys).  s_tot: 4 words of LDS,
// s_out: 2 words.
__device__ void block_rank_bin(const uint32_t* h, uint32_t need, uint32_t* s_tot, int32_t* s_out, int* digit,
                               uint32_t* nneed) {
  constexpr int PER = kBoundBins / kDenseThreads;  // bins per thread
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_out[0] = -1;
  uint32_t local = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) local += h[PER * tid + j];
  uint32_t incl = local;  // keys in this thread's bins and every higher one, within the wavefront
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_down(incl, o);
    if (lane + o < 64) incl += t;
  }
  if (lane == 0) s_tot[wave] = incl;
  __syncthreads();
  for (int w = wave + 1; w < kDenseThreads / 64; ++w) incl += s_tot[w];
  uint32_t above = incl - local;
  if (above < need && need <= incl) {
    for (int j = PER - 1; j >= 0; --j) {
      const uint32_t c = h[PER * tid + j];
      if (above < need && need <= above + c) {
        s_out[0] = PER * tid + j;
        s_out[1] = (int32_t)(need - above);
      }
      above += c;
    }
  }
  __syncthreads();
  *digit = s_out[0];
  *nneed = (uint32_t)s_out[1];
  __syncthreads();
}

// The first seeds of a search: seed[q] = the bound of the kappa-th best;
// seed_opt (may be null): max(seed[q], bound of the rank_opt-th best), the next
// level's optimistic seed.  One workgroup per query; a row with fewer than a
// rank's finite scores gives that rank no bound (-inf).
__global__ __launch_bounds__(kDenseThreads) void k_dense_select(const float* __restrict__ dense, int64_t m,
                                                                int64_t ns, int kappa, float* __restrict__ seed,
                                                                float* __restrict__ seed_opt, int rank_opt) {
  __shared__ uint32_t hist[2][kBoundBins];
  __shared__ uint32_t s_tot[4];
  __shared__ int32_t s_out[2];
  __shared__ int s_valid;
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x;
  if (q >= m) return;
  const float* row = dense + q * ns;
  const int nr = seed_opt ? 2 : 1;
  const uint32_t rank[2] = {(uint32_t)kappa, (uint32_t)rank_opt};
  constexpr int kUn = 8;  // loads in flight per thread
  for (int b = tid; b < 2 * kBoundBins; b += kDenseThreads) (&hist[0][0])[b] = 0;
  if (tid == 0) s_valid = 0;
  __syncthreads();
  // first pass: the top 11 bits of every key, and the finite scores
  int valid = 0;
  for (int64_t i0 = tid; i0 < ns; i0 += (int64_t)kDenseThreads * kUn) {
    float v[kUn];
#pragma unroll
    for (int u = 0; u < kUn; ++u) v[u] = i0 + kDenseThreads * u < ns ? row[i0 + kDenseThreads * u] : -INFINITY;
#pragma unroll
    for (int u = 0; u < kUn; ++u) {
      valid += v[u] != -INFINITY;
      if (i0 + kDenseThreads * u < ns) atomicAdd(&hist[0][order_f32(v[u]) >> 21], 1u);
    }
  }
  for (int o = 32; o > 0; o >>= 1) valid += __shfl_xor(valid, o);
  if ((tid & 63) == 0) atomicAdd(&s_valid, valid);
  __syncthreads();
  const int nvalid = s_valid;
  int d0[2] = {-1, -1};
  uint32_t need[2] = {0, 0};
  for (int r = 0; r < nr; ++r)
    if ((int)rank[r] <= nvalid) block_rank_bin(hist[0], rank[r], s_tot, s_out, &d0[r], &need[r]);
  // second pass: the next 11 bits of the keys under each rank's top bits
  for (int b = tid; b < 2 * kBoundBins; b += kDenseThreads) (&hist[0][0])[b] = 0;
  __syncthreads();
  if (d0[0] >= 0 || d0[1] >= 0) {
    for (int64_t i0 = tid; i0 < ns; i0 += (int64_t)kDenseThreads * kUn) {
      float v[kUn];
#pragma unroll
      for (int u = 0; u < kUn; ++u) v[u] = i0 + kDenseThreads * u < ns ? row[i0 + kDenseThreads * u] : -INFINITY;
#pragma unroll
      for (int u = 0; u < kUn; ++u) {
        const uint32_t k = order_f32(v[u]);
        const bool in = i0 + kDenseThreads * u < ns;
#pragma unroll
        for (int r = 0; r < 2; ++r)
          if (in && (int)(k >> 21) == d0[r]) atomicAdd(&hist[r][(k >> 10) & (kBoundBins - 1)], 1u);
      }
    }
  }
  __syncthreads();
  float tau[2] = {-INFINITY, -INFINITY};
  for (int r = 0; r < nr; ++r) {
    if (d0[r] < 0) continue;
    int d1;
    uint32_t rest;
    block_rank_bin(hist[r], need[r], s_tot, s_out, &d1, &rest);
    const float t = unorder_f32(((uint32_t)d0[r] << 21) | ((uint32_t)d1 << 10));  // the smallest key with these 22 bits
    tau[r] = t != t ? -INFINITY : t;  // a prefix below every finite score's key
  }
  if (tid == 0) {
    seed[q] = tau[0];
    if (seed_opt) seed_opt[q] = fmaxf(tau[0], tau[1]);
  }
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
static_assert(kMaxKappa <= kSelWin / 2, "a select window holds the kappa kept keys and as many new ones");

// bitonic sort, descending, of the first `size` entries (a power of two) of
// key[] in LDS by every thread of the workgroup (nthreads threads)
template <typename T>
__device__ void block_sort_desc(T* key, int size, int nthreads) {
  for (int k = 2; k <= size; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < size; i += nthreads) {
        const int l = i ^ j;
        if (l > i) {
          const bool desc = (i & k) == 0;
          const T x = key[i], y = key[l];
          if (desc ? (x < y) : (x > y)) {
            key[i] = y;
            key[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__host__ __device__ inline int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// seed_opt (sample levels, may be null): also the kappa_opt-th best score, an
// optimistic seed for the next level (see run_scan).
template <bool FINAL>
__global__ __launch_bounds__(256) void k_select(const uint64_t* __restrict__ buf, const int32_t* __restrict__ cnt,
                                                int R, int cap, int kappa, const int32_t* __restrict__ ids,
                                                float* __restrict__ seed, int32_t* __restrict__ out_ids,
                                                float* __restrict__ out_scores, float* __restrict__ seed_opt,
                                                int kappa_opt) {
  __shared__ uint64_t keys[kSelWin];
  __shared__ int32_t pre[kMaxLists + 1];
  __shared__ uint64_t stage[kMaxKappa];
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
    // each thread gathers up to kSelWin / 256 keys: every list position is found
    // first, then all the loads are issued together (one memory latency per
    // window instead of one per key)
    constexpr int kPer = kSelWin / 256;
    uint64_t kv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int f = tid + 256 * j;
      kv[j] = 0;
      if (f < wn) {
        const int g = (int)(w0 + f);
        int lo = 0, hi = R - 1;  // list holding flat index g: last L with pre[L] <= g
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pre[mid] <= g) lo = mid; else hi = mid - 1;
        }
        kv[j] = buf[(q * R + lo) * (int64_t)cap + (g - pre[lo])];
      }
    }
    if (FINAL) {  // re-key by original id (the ids are loaded together as well)
      int32_t idv[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int f = tid + 256 * j;
        idv[j] = f < wn ? ids[0xFFFFFFFFu - (uint32_t)kv[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        kv[j] = (kv[j] & 0xFFFFFFFF00000000ull) | (uint64_t)(0xFFFFFFFFu - (uint32_t)idv[j]);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int f = tid + 256 * j;
      if (f < wn) keys[kept + f] = kv[j];
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
    if (kept < kappa) {  // fewer than kappa candidates: no exact kappa-th best
      // all the level's candidates are kept: the kappa_opt-th best is exact when
      // there are that many
      float opt = -INFINITY;
      if (seed_opt && kept >= kappa_opt) opt = key_score(block_kth(keys, kept, kappa_opt, sel));
      if (seed_opt && tid == 0) seed_opt[q] = fmaxf(seed[q], opt);
      return;
    }
    // the kappa-th best is the smallest kept key
    uint64_t mn = ~0ull;
    for (int i = tid; i < kept; i += 256) mn = std::min(mn, keys[i]);
    for (int o = 32; o > 0; o >>= 1) mn = std::min(mn, (uint64_t)__shfl_xor(mn, o));
    if (lane == 0) stage[wave] = mn;
    __syncthreads();
    float opt = -INFINITY;
    if (seed_opt) opt = key_score(block_kth(keys, kept, kappa_opt, sel));  // every thread takes part
    if (tid == 0) {
      const uint64_t m4 = std::min(std::min(stage[0], stage[1]), std::min(stage[2], stage[3]));
      const float sd = fmaxf(seed[q], key_score(m4));
      seed[q] = sd;
      if (seed_opt) seed_opt[q] = fmaxf(sd, opt);
    }
    return;
  }
  // bitonic sort of the kept keys, descending (padding keys are 0)
  const int sn = pow2_at_least(kappa);
  for (int i = tid; i < sn; i += 256) stage[i] = i < kept ? keys[i] : 0;
  __syncthreads();
  block_sort_desc(stage, sn, 256);
  for (int i = tid; i < kappa; i += 256) {
    const uint64_t k = stage[i];
    out_ids[q * kappa + i] = (int32_t)key_id(k);
    out_scores[q * kappa + i] = key_score(k);
  }
}

// whole_lists: one query block per workgroup (no tile ring), whose wavefronts
// stage a whole list in a compaction -- for kappa beyond a ring shape's staging
// wave_mul: workgroups per query group of a many-query scan, as a multiple of
// the base count (shorter row ranges keep the workgroups that share a range in
// step, so their tiles stay in L2; each range costs one list per query)
Shape choose_shape(int fmt, int dp, int64_t m, int64_t rows, int C, const Tuning& tu, bool whole_lists = false,
                   int wave_mul = 1) {
  Shape sh;
  const int qpw_override = tu.qpw;
  if (whole_lists) {
    sh.nb = m <= 32 ? 1 : 2;
    sh.shared = true;
  } else if (qpw_override > 0) {
    sh.nb = std::max(1, std::min(4, qpw_override / 32));
    sh.shared = m <= sh.nb * 32;
  } else if (m <= 32) {
    sh.shared = true; sh.nb = 1;
  } else if (m <= 64) {
    sh.shared = true; sh.nb = 2;
  } else {
    sh.shared = false; sh.nb = 2;  // two wavefronts per SIMD on the LDS ring (see launch_one)
  }
  if (sh.shared && sh.nb > 2) sh.nb = 2;
  if (!sh.shared && sh.nb < 2) sh.nb = 2;
  if (fmt == GV_FP32) sh.nb = 1;
  if (dp > 160 && sh.nb > 2) sh.nb = 2;  // keeps the query views of the longest rows in registers
  sh.nqb = (m + 32 * sh.nb - 1) / (32 * sh.nb);
  const int64_t ntiles = rows / kRows + C;
  // about 1024 wavefronts (one per SIMD) when the query blocks share a workgroup's
  // rows, 2048 times wave_mul otherwise (several rounds of workgroups, which
  // even out ranges that hold many survivors); at least 4 tiles per range
  const int64_t waves = sh.shared ? 1024 : 2048LL * wave_mul;
  int64_t R = tu.splits > 0 ? tu.splits : std::max<int64_t>(1, waves / sh.nqb);
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

gv_status dispatch_fmt_queue(int fmt, int dp, const Shape& sh, int grid, const ScoreArgs* args, const int64_t* off,
                             int ncoll, int* head, hipStream_t st) {
  switch (fmt) {
    case GV_FP32: return dispatch_scan_queue<GV_FP32>(dp, sh, grid, args, off, ncoll, head, st);
    case GV_FP16: return dispatch_scan_queue<GV_FP16>(dp, sh, grid, args, off, ncoll, head, st);
    case GV_BF16: return dispatch_scan_queue<GV_BF16>(dp, sh, grid, args, off, ncoll, head, st);
    default: return dispatch_scan_queue<GV_FP8_E4M3>(dp, sh, grid, args, off, ncoll, head, st);
  }
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
// The cascade's strides, sparsest sample first, ending with the full scan
// (stride 1): powers of `step` whose samples hold at least 8 kappa rows.
// Small batches step by 64 when that still leaves a filtering level between
// the dense sample and the full scan: their scans are bound by HBM, so a
// sample level costs its launches and select more than its rows, and fewer,
// wider steps win even though the full scan starts from a looser seed.  Large
// batches (and databases too small for two 64-fold steps, where the full scan
// would start from the dense sample's bound) step by 16, which keeps the full
// scan's survivors few.
constexpr int64_t kCoarseCascadeM = 256;
std::vector<int64_t> cascade(int64_t n, int kappa, int64_t m) {
  auto ladder = [&](int64_t step) {
    std::vector<int64_t> s{1};
    int64_t top = 0;
    for (int64_t stride = step; n / stride >= 8LL * kappa && stride <= (1LL << 24); stride *= step) top = stride;
    for (int64_t stride = step; stride <= top; stride *= step) s.insert(s.begin(), stride);
    return s;
  };
  if (m <= kCoarseCascadeM) {
    std::vector<int64_t> s = ladder(64);
    if (s.size() >= 3) return s;
  }
  return ladder(16);
}

}  // namespace

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

// a list capacity every launch shape accepts for kappa: a list is checked for
// overflow at least every 13 tiles and takes at most 32 keys per tile (each
// plan checks its own shapes: list_limit > kappa)
int min_list_cap(int kappa) { return kappa + kRows * 13 + 1; }

namespace {

// Launch plan of S2/S3 for one (index, m, kappa): cascade levels, their
// shapes, and the scratch they need.
struct ScanPlan {
  std::vector<int64_t> levels;
  std::vector<Shape> shapes;
  std::vector<ScanLimits> limits;
  bool has_dense = false;
  uint64_t keys = 0;  // list slots of the scratch (m x Rmax x cap)
  int Rmax = 1;
  int64_t ns = 0;
  int cap = kCap;
  int dp = 0;  // padded length of the scanned leading part of each row
  // the full scan starts from an optimistic seed, the kappa_opt-th best score
  // of the last sample level, and a repair pass rescans the rare queries for
  // which it kept fewer than kappa keys (see run_scan)
  bool optimistic = false;
  int kappa_opt = 0;                 // rank of the full scan's optimistic seed
  std::vector<int> next_rank;        // per level: rank of the optimistic seed it gives the next level
  size_t off_buf = 0, off_cnt = 0, off_seed = 0, off_dense = 0, off_seed_opt = 0, off_rescan = 0, bytes = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// the k_scan instantiation a shape launches, described on the host
template <int FMT>
ScanLimits limits_fmt(int dp, const Shape& sh) {
  constexpr int km = MfmaOp<FMT>::KM;
  switch (dp / km) {
    case 32 / km: return limits_for_shape<FMT, 32 / km>(sh);
    case 64 / km: return limits_for_shape<FMT, 64 / km>(sh);
    case 128 / km: return limits_for_shape<FMT, 128 / km>(sh);
    case 160 / km: return limits_for_shape<FMT, 160 / km>(sh);
    case 192 / km: return limits_for_shape<FMT, 192 / km>(sh);
    default: return limits_for_shape<FMT, 256 / km>(sh);
  }
}
ScanLimits scan_limits(int fmt, int dp, const Shape& sh) {
  switch (fmt) {
    case GV_FP32: return limits_fmt<GV_FP32>(dp, sh);
    case GV_FP16: return limits_fmt<GV_FP16>(dp, sh);
    case GV_BF16: return limits_fmt<GV_BF16>(dp, sh);
    default: return limits_fmt<GV_FP8_E4M3>(dp, sh);
  }
}

// The launch plan of S2/S3 from the index dimensions alone: n rows stored as
// n_pad (segments padded to whole tiles), C clusters, format, stored padded
// length dps, leading length dp_search scanned.
gv_status plan_scan_dims(int64_t n, int64_t n_pad, int C, int fmt, int dps, int d_search, int64_t m, int kappa,
                         ScanPlan* p, uint64_t list_budget = kListBudgetLarge) {
  p->dp = pad_dim(d_search);
  if (p->dp > dps || p->dp > 256) {
    set_error("the scan reads at most the leading 256 stored coordinates (padded), and no more than the index stores");
    return GV_EUNSUPPORTED;
  }
  const Tuning tu = effective_tuning(fmt, p->dp, m, n);
  p->levels = cascade(n, kappa, m);
  p->has_dense = p->levels.size() > 1;
  const int64_t ntiles = n_pad / kRows;
  // the shapes of every level for a list capacity and a workgroup multiple;
  // GV_OK when every filtering level leaves a list room above kappa
  auto build = [&](int cap, int wave_mul) -> gv_status {
    p->cap = cap;
    p->shapes.clear();
    p->limits.clear();
    p->Rmax = 1;
    for (size_t li = 0; li < p->levels.size(); ++li) {
      const int64_t s = p->levels[li];
      const int64_t rows = (ntiles + s - 1) / s * kRows;
      Shape sh = choose_shape(fmt, p->dp, m, rows, C, tu, false, wave_mul);
      ScanLimits lm = scan_limits(fmt, p->dp, sh);
      const bool dense = p->has_dense && li == 0;  // the dense scan writes no lists
      if (!dense) {
        // a list is compacted once it holds more than lim keys and may then grow
        // by 32 keys per tile for U + 1 tiles before the next check: the staging
        // (CAPL) and the list (cap) must hold that, and a compaction to the kappa
        // best must leave room (lim > kappa)
        auto limit = [&](const ScanLimits& l) { return std::min(p->cap, l.CAPL) - kRows * (l.U + 1); };
        if (limit(lm) <= kappa && !sh.shared) {  // a shape that stages whole lists
          sh = choose_shape(fmt, p->dp, m, rows, C, tu, true, wave_mul);
          lm = scan_limits(fmt, p->dp, sh);
        }
        p->Rmax = std::max(p->Rmax, sh.R);
        if (limit(lm) <= kappa) {
          set_error("kappa too large for the candidate lists of this launch shape (reduce kappa or raise the list cap)");
          return GV_EUNSUPPORTED;
        }
      }
      p->shapes.push_back(sh);
      p->limits.push_back(lm);
    }
    return GV_OK;
  };
  if (tu.cap > 0 && (tu.cap <= kappa || tu.cap > kCap)) {
    set_error("candidate list capacity must lie in (kappa, 2048]");
    return GV_EINVAL;
  }
  bool chosen = false;
  if (tu.cap == 0 && tu.splits == 0) {
    // automatic: the most workgroups (up to eight times the base count) with
    // the smallest list capacity (at least 512) whose lists fit in kListBudget.
    // Batches large enough that sixteen times the base count still gives at
    // most 1024 row ranges (m >= 2048 on 10M rows) first try that shape, with
    // lists up to list_budget: 3% faster at m = 2048 and 4096 than the eightfold
    // count, while more ranges were slower at m = 1024
    auto fits = [&](int cap, uint64_t budget) { return (uint64_t)m * p->Rmax * cap * sizeof(uint64_t) <= budget; };
    chosen = build(512, 16) == GV_OK && p->Rmax <= 1024 && fits(512, list_budget);
    for (int mul = 8; mul >= 1 && !chosen; mul /= 2)
      for (int cap = 512; cap <= kCap && !chosen; cap *= 2)
        chosen = build(cap, mul) == GV_OK && fits(cap, kListBudget);
    clear_error();
  }
  if (!chosen) GV_TRY(build(tu.cap > 0 ? tu.cap : kCap, 1));
  p->ns = p->has_dense ? ((ntiles + p->levels[0] - 1) / p->levels[0]) * kRows : 0;
  // Optimistic seeds, when the level before the full scan filters: every
  // filtering level starts from a higher-ranked score of the level before.  If
  // a sample holds each row of the next level with probability f, the number of
  // its rows among a query's kappa - 1 best there is about Binomial(kappa, f);
  // the kappa_opt-th best sample score exceeds the query's kappa-th best only if
  // that count reaches kappa_opt = f kappa + 6 sqrt(f kappa) + 6 (six standard
  // deviations, plus room for small kappa).  About kappa_opt / f keys then
  // survive instead of kappa / f.  The full scan's repair pass keeps its result
  // exact; a sample level that keeps fewer than kappa keys leaves the exact seed
  // of the level before in place.
  p->optimistic = false;
  p->kappa_opt = 0;
  p->next_rank.assign(p->levels.size(), 0);
  const int ov = tuned_optimism();
  const size_t nl = p->levels.size();
  if (nl >= 3 && ov >= 0) {
    // the rank whose score, taken in a sample of fraction f of the next level,
    // leaves at least `need` rows of that level above it (six standard deviations)
    auto rank_for = [&](int need, size_t li) {
      const double mu = (double)need * (double)p->levels[li + 1] / (double)p->levels[li];
      return ov > 0 ? ov : (int)std::ceil(mu + 6.0 * std::sqrt(mu) + 6.0);
    };
    const int ko = rank_for(kappa, nl - 2);
    if (ko < kappa) {
      p->optimistic = true;
      p->kappa_opt = ko;
      // the level before the full scan gives it rank ko; an earlier sample level
      // only needs its successor to keep the rank that successor passes on
      int need = ko;
      p->next_rank[nl - 2] = ko;
      for (size_t li = nl - 2; li-- > 0;) {  // earlier sample levels, the dense one (level 0) included
        const int r = std::min(rank_for(need, li), kappa);
        p->next_rank[li] = r;
        need = r;
      }
    }
  }
  const uint64_t keys = (uint64_t)m * p->Rmax * p->cap;
  if (keys >= (1ull << 32)) {  // list slots are staged as 32-bit indices
    set_error("search batch too large for the candidate lists (reduce m)");
    return GV_EUNSUPPORTED;
  }
  p->keys = keys;
  size_t o = 0;
  p->off_buf = o;   o = align256(o + sizeof(uint64_t) * keys);
  p->off_cnt = o;   o = align256(o + sizeof(int32_t) * m * p->Rmax);
  p->off_seed = o;  o = align256(o + (p->has_dense ? sizeof(float) * m : 0));
  p->off_dense = o; o = align256(o + (p->has_dense ? sizeof(float) * m * p->ns : 0));
  p->off_seed_opt = o; o = align256(o + (p->optimistic ? sizeof(float) * m : 0));
  p->off_rescan = o;   o = align256(o + (p->optimistic ? sizeof(float) * m : 0));
  p->bytes = o;
  return GV_OK;
}

gv_status plan_scan(const gv_index* idx, int64_t m, int kappa, ScanPlan* p, int d_search = 0,
                    uint64_t list_budget = kListBudgetLarge) {
  return plan_scan_dims(idx->n_rows, idx->n_pad, idx->C, idx->fmt, idx->dp, d_search > 0 ? d_search : idx->d, m,
                        kappa, p, list_budget);
}

// views made inside the scan (Algorithm 3) instead of qhat/t
struct LazyViews {
  const double* A;
  const float* Q;
  int d, D, ds;
};

// Which part of the cascade run_scan issues: all of it; everything but the
// full scan and its select (the full scan's arguments and shape are returned
// instead, for a persistent launch that scans several searches); or only the
// final select after such a launch.
enum class Part { All, Prefix, Suffix };

gv_status run_scan(const gv_index* idx, const ScanPlan& p, uint8_t* ws, const void* qhat, const float* t, int64_t m,
                   int kappa, int32_t* cand_ids, float* cand_scores, hipStream_t st, const LazyViews* lazy = nullptr,
                   Part part = Part::All, ScoreArgs* last_args = nullptr, Shape* last_shape = nullptr) {
  uint64_t* buf = (uint64_t*)(ws + p.off_buf);
  int32_t* cnt = (int32_t*)(ws + p.off_cnt);
  float* seed = p.has_dense ? (float*)(ws + p.off_seed) : nullptr;
  float* dense = p.has_dense ? (float*)(ws + p.off_dense) : nullptr;
  float* seed_opt = p.optimistic ? (float*)(ws + p.off_seed_opt) : nullptr;
  float* rescan = p.optimistic ? (float*)(ws + p.off_rescan) : nullptr;
  const int fmt = idx->fmt;

  ScoreArgs args{};
  Shape sh_cur{};
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
  args.dp = p.dp;
  args.dps = idx->dp;
  args.kappa = kappa;
  args.cap = p.cap;
  if (lazy) {
    args.lazy_A = lazy->A;
    args.lazy_Q = lazy->Q;
    args.lazy_d = lazy->d;
    args.lazy_D = lazy->D;
    args.lazy_ds = lazy->ds;
  }
  auto dispatch = [&](bool dense) -> gv_status {
    if (lazy) return dense ? dispatch_scan_lazy<kDense>(sh_cur, args, st) : dispatch_scan_lazy<kFilter>(sh_cur, args, st);
    return dense ? dispatch_fmt<kDense>(fmt, p.dp, sh_cur, args, st) : dispatch_fmt<kFilter>(fmt, p.dp, sh_cur, args, st);
  };
  // after the optimistic full scan (args and sh_cur set for it): queries that
  // kept fewer than kappa keys are rescanned from the exact seed
  auto repair = [&]() -> gv_status {
    hipLaunchKernelGGL(k_repair_prep, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, cnt, sh_cur.R, m, kappa, seed,
                       seed_opt, rescan);
    const float* s0 = args.seed;
    args.seed = rescan;
    args.repair = 1;
    const gv_status r = dispatch(false);
    args.seed = s0;
    args.repair = 0;
    return r;
  };

  gv_status s = GV_OK;
  for (size_t li = 0; li < p.levels.size() && s == GV_OK; ++li) {
    const Shape& sh = p.shapes[li];
    sh_cur = sh;
    const bool last = li + 1 == p.levels.size();
    // filtering levels start from the optimistic seed of the level before (the
    // full scan repairs what it misses; a sample level that keeps fewer than
    // kappa keys leaves the exact seed as it was)
    args.seed = li == 0 ? nullptr : (p.optimistic ? seed_opt : seed);
    args.R = sh.R;
    args.nqb = (int)sh.nqb;
    args.stride = (int)p.levels[li];
    args.xcd_map = sh.xcd_map;
    if (part == Part::Suffix && !last) continue;
    if (part == Part::Prefix && last) {  // the full scan runs elsewhere, from these arguments
      if (sh.R > p.Rmax || p.levels[li] != 1 || lazy) {
        set_error("internal: candidate scratch smaller than the launch");
        return GV_EDEVICE;
      }
      args.xcd_map = 0;  // a queue hands pieces to workgroups in any order
      if (last_args) *last_args = args;
      if (last_shape) *last_shape = sh;
      break;
    }
    if (part == Part::Suffix) {
      if (p.optimistic) s = repair();
      if (s != GV_OK) break;
      hipLaunchKernelGGL(k_select<true>, dim3((unsigned)m), dim3(256), 0, st, buf, cnt, sh.R, p.cap, kappa, idx->ids,
                         seed, cand_ids, cand_scores, (float*)nullptr, 0);
      break;
    }
    if (p.has_dense && li == 0) {
      s = dispatch(true);
      if (s == GV_OK)
        hipLaunchKernelGGL(k_dense_select, dim3((unsigned)m), dim3(kDenseThreads), 0, st, dense, m, p.ns, kappa,
                           seed, p.optimistic ? seed_opt : (float*)nullptr, p.next_rank[0]);
      continue;
    }
    if (sh.R > p.Rmax) {  // scratch must cover every list the launch writes
      set_error("internal: candidate scratch smaller than the launch");
      return GV_EDEVICE;
    }
    if (last) profile_mark(st, 0, true);
    s = dispatch(false);
    if (last) profile_mark(st, 0, false);
    if (s != GV_OK) break;
    if (last) {
      if (p.optimistic) s = repair();
      if (s != GV_OK) break;
      profile_mark(st, 1, true);
      hipLaunchKernelGGL(k_select<true>, dim3((unsigned)m), dim3(256), 0, st, buf, cnt, sh.R, p.cap, kappa, idx->ids,
                         seed, cand_ids, cand_scores, (float*)nullptr, 0);
      profile_mark(st, 1, false);
    } else {
      // a sample level also yields the optimistic seed of the next level
      hipLaunchKernelGGL(k_select<false>, dim3((unsigned)m), dim3(256), 0, st, buf, cnt, sh.R, p.cap, kappa,
                         idx->ids, seed, (int32_t*)nullptr, (float*)nullptr, p.optimistic ? seed_opt : (float*)nullptr,
                         p.next_rank[li]);
    }
  }
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace

gv_status scan_plan_describe(int64_t n, int64_t n_pad, int C, int fmt, int d, int d_search, int64_t m, int kappa,
                             gv_scan_level* levels, int max_levels, int* n_levels, int64_t* list_keys,
                             int64_t* scratch_bytes) {
  ScanPlan p;
  GV_TRY(plan_scan_dims(n, n_pad, C, fmt, pad_dim(d), d_search > 0 ? d_search : d, m, kappa, &p));
  const int nl = (int)p.levels.size();
  if (n_levels) *n_levels = nl;
  if (list_keys) *list_keys = (int64_t)p.keys;
  if (scratch_bytes) *scratch_bytes = (int64_t)p.bytes;
  for (int li = 0; li < nl && li < max_levels && levels; ++li) {
    const Shape& sh = p.shapes[li];
    const ScanLimits& lm = p.limits[li];
    gv_scan_level& o = levels[li];
    o.stride = p.levels[li];
    o.dense = (p.has_dense && li == 0) ? 1 : 0;
    o.ranges = sh.R;
    o.grid = sh.grid;
    o.query_blocks = sh.nqb;
    o.queries_per_wave = 32 * lm.nb;
    o.shared = sh.shared ? 1 : 0;
    o.xcd_map = sh.xcd_map;
    o.tile_ring = lm.ring ? 1 : 0;
    o.workgroups_per_cu = lm.occupancy;
    o.check_every = lm.U;
    o.staging = lm.CAPL;
    o.list_cap = p.cap;
    o.list_limit = std::min(p.cap, lm.CAPL) - kRows * (lm.U + 1);
    o.rows_per_level = (n_pad / kRows + p.levels[li] - 1) / p.levels[li] * kRows;
  }
  return GV_OK;
}

gv_status score_topk_impl(const gv_index* idx, const void* qhat, const float* t, int64_t m, int kappa,
                          int32_t* cand_ids, float* cand_scores, hipStream_t st, int d_search) {
  if (m == 0) return GV_OK;
  keep_pool(idx->device);
  ScanPlan p;
  GV_TRY(plan_scan(idx, m, kappa, &p, d_search));
  uint8_t* ws = nullptr;
  if (dev_malloc_async((void**)&ws, std::max<size_t>(p.bytes, 256), st) != hipSuccess) {
    set_error("search scratch allocation failed");
    return GV_ENOMEM;
  }
  const gv_status s = run_scan(idx, p, ws, qhat, t, m, kappa, cand_ids, cand_scores, st);
  (void)hipFreeAsync(ws, st);
  return s;
}

// ---------------------------------------------------------------------------- whole search
// Scratch of one search (S1 views and scales, S2/S3 lists, candidates), carved
// from one workspace so the sequence runs without allocations.
gv_status search_plan(const gv_model* model, const gv_index* idx, int64_t m, int kappa, SearchPlan* sp,
                      int d_search, bool stored, uint64_t list_budget) {
  ScanPlan p;
  GV_TRY(plan_scan(idx, m, kappa, &p, d_search, list_budget));
  if (!stored && !idx->X) {
    set_error("the index keeps no full-dimension vectors: rerank from the stored vectors");
    return GV_EINVAL;
  }
  sp->d_search = d_search;
  sp->stored = stored;
  sp->list_budget = list_budget;
  const size_t C = idx->C, dp = idx->dp, eb = fmt_bytes(view_fmt(idx->fmt));
  size_t o = 0;
  sp->off_t = o;    o = align256(o + sizeof(float) * m * C);
  sp->off_qc = o;   o = align256(o + sizeof(float) * m * C * dp);
  sp->off_qhat = o; o = align256(o + eb * m * C * p.dp);
  sp->off_cand = o; o = align256(o + sizeof(int32_t) * m * kappa);
  sp->off_csc = o;  o = align256(o + sizeof(float) * m * kappa);
  // the scan's scratch is free before the first level and after the final
  // select: S1's partial products and S4's scores use it then
  const size_t region = std::max(p.bytes, proj_split_bytes(m, (int64_t)model->C * model->d, model->D));
  sp->off_scan = o; o = align256(o + region);
  sp->scan_bytes = p.bytes;
  sp->region_bytes = region;
  sp->bytes = std::max<size_t>(o, 256);
  return GV_OK;
}

gv_status search_run(const gv_model* model, const gv_index* idx, const float* Q, int64_t m, int k, int kappa,
                     int32_t* out_ids, float* out_scores, const SearchPlan& sp, void* workspace, hipStream_t st) {
  if (m == 0) return GV_OK;
  uint8_t* ws = (uint8_t*)workspace;
  ScanPlan p;
  GV_TRY(plan_scan(idx, m, kappa, &p, sp.d_search, sp.list_budget));
  if (p.bytes > sp.scan_bytes) {  // the workspace was sized for another plan (tuning changed in between)
    set_error("internal: the search plan changed after its workspace was sized");
    return GV_EDEVICE;
  }
  float* t = (float*)(ws + sp.off_t);
  float* qc = (float*)(ws + sp.off_qc);
  void* qhat = ws + sp.off_qhat;
  int32_t* cand = (int32_t*)(ws + sp.off_cand);
  float* csc = (float*)(ws + sp.off_csc);
  GV_TRY(project_impl(model, idx->fmt, Q, m, qc, t, qhat, st, sp.d_search, ws + sp.off_scan, sp.region_bytes));
  GV_TRY(run_scan(idx, p, ws + sp.off_scan, qhat, t, m, kappa, cand, csc, st));
  if (sp.stored)
    GV_TRY(rerank_stored_impl(idx, qc, m, cand, kappa, k, out_ids, out_scores, st));
  else
    GV_TRY(rerank_impl(idx, Q, m, cand, kappa, k, out_ids, out_scores, st, ws + sp.off_scan, sp.region_bytes));
  return GV_OK;
}

// The search with the lazy inner product (Algorithm 3): no S1 pass; the scan
// projects q_c = A_c q for the cluster it visits, in each work item.  FP16
// storage, padded length 160, batches small enough for one shared query block
// whose eager projection runs the same arithmetic (m <= 16).
gv_status search_lazy_impl(const gv_model* model, const gv_index* idx, const float* Q, int64_t m, int k, int kappa,
                           int32_t* out_ids, float* out_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  if (idx->fmt != GV_FP16 || idx->dp != 160 || m > kSmallM || !idx->X) {
    set_error("lazy search: needs FP16 storage, a padded reduced length of 160, m <= 16 and an index that keeps X");
    return GV_EUNSUPPORTED;
  }
  ScanPlan p;
  GV_TRY(plan_scan(idx, m, kappa, &p));
  for (const Shape& sh : p.shapes)
    if (!sh.shared || sh.nb != 1) {
      set_error("lazy search: the launch shape must be one shared block of 32 queries (no qpw override)");
      return GV_EUNSUPPORTED;
    }
  keep_pool(idx->device);
  const size_t off_cand = align256(p.bytes), off_csc = align256(off_cand + sizeof(int32_t) * m * kappa);
  const size_t bytes = align256(off_csc + sizeof(float) * m * kappa);
  uint8_t* ws = nullptr;
  if (dev_malloc_async((void**)&ws, bytes, st) != hipSuccess) {
    set_error("search scratch allocation failed");
    return GV_ENOMEM;
  }
  LazyViews lv{model->A, Q, model->d, model->D, model->d};
  int32_t* cand = (int32_t*)(ws + off_cand);
  float* csc = (float*)(ws + off_csc);
  gv_status s = run_scan(idx, p, ws, nullptr, nullptr, m, kappa, cand, csc, st, &lv);
  if (s == GV_OK) s = rerank_impl(idx, Q, m, cand, kappa, k, out_ids, out_scores, st, ws, p.bytes);
  (void)hipFreeAsync(ws, st);
  return s;
}

// ---------------------------------------------------------------------------- batched executor
// Several searches (collections) as one launch sequence on `org`, for capture
// into one graph: the projections and cascade levels of every search run as
// branches on the side streams; then the full-database scans of all searches
// run as persistent queue kernels, one per kernel instantiation, whose
// workgroups pull (search, piece) items until every search's scan is done;
// then the final selects and reranks run as branches again.  Each search has
// its own workspace (its lists live from its cascade to its final select).
gv_status batched_run(std::vector<BatchEntry>& e, int k, int kappa, hipStream_t org, hipStream_t* side, int nside,
                      hipEvent_t fork, hipEvent_t* join, uint8_t* qmem, size_t qbytes, int n_cu,
                      std::vector<uint8_t>* upload) {
  const int ne = (int)e.size();
  // classes: searches whose full scans share one kernel instantiation
  struct Cls {
    int fmt, dp, nb;
    bool shared;
    std::vector<int> members;
  };
  std::vector<Cls> cls;
  std::vector<ScanPlan> plans(ne);
  for (int i = 0; i < ne; ++i) {
    GV_TRY(plan_scan(e[i].idx, e[i].m, kappa, &plans[i], e[i].plan.d_search, e[i].plan.list_budget));
    const Shape& sh = plans[i].shapes.back();
    const int fmt = e[i].idx->fmt, dp = plans[i].dp;
    int c = -1;
    for (int j = 0; j < (int)cls.size(); ++j)
      if (cls[j].fmt == fmt && cls[j].dp == dp && cls[j].nb == sh.nb && cls[j].shared == sh.shared) c = j;
    if (c < 0) {
      cls.push_back(Cls{fmt, dp, sh.nb, sh.shared, {}});
      c = (int)cls.size() - 1;
    }
    cls[c].members.push_back(i);
  }
  // queue memory: per class an argument array and a piece offset array, then
  // one head counter per class
  size_t o = 0;
  std::vector<size_t> off_args(cls.size()), off_off(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) {
    off_args[c] = o; o = align256(o + sizeof(ScoreArgs) * cls[c].members.size());
    off_off[c] = o;  o = align256(o + sizeof(int64_t) * (cls[c].members.size() + 1));
  }
  const size_t off_heads = o;
  o = align256(o + sizeof(int) * cls.size());
  if (o > qbytes) {
    set_error("internal: batched queue memory too small");
    return GV_EDEVICE;
  }
  upload->assign(off_heads, 0);

  // branches to streams: longest first onto the least loaded stream, by a rough
  // time model of each search's branch (a launch latency per kernel, the S1
  // FP64 product, the sample levels' reads and matrix-core work, the rerank's
  // gathers)
  auto assign = [&](const std::vector<double>& cost) {
    std::vector<int> order(ne), to(ne);
    for (int i = 0; i < ne; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(nside, 0.0);
    for (int i : order) {
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      to[i] = j;
      load[j] += cost[i];
    }
    return to;
  };
  std::vector<double> c_pre(ne), c_suf(ne);
  for (int i = 0; i < ne; ++i) {
    const gv_index* ix = e[i].idx;
    const double m = (double)e[i].m, C = ix->C, d = ix->d, D = ix->D, dp = plans[i].dp;
    const double eb = ix->fmt == GV_FP32 ? 4.0 : (ix->fmt == GV_FP8_E4M3 ? 1.0 : 2.0);
    double t = 15e-6 * (2.0 + 2.0 * (double)(plans[i].levels.size() - 1)) + 2.0 * m * C * d * D / 35e12;
    for (size_t li = 0; li + 1 < plans[i].levels.size(); ++li) {
      const double rows = (double)ix->n_rows / (double)plans[i].levels[li];
      t += std::max(2.0 * m * rows * dp / 1e15, rows * dp * eb / 5e12);
    }
    c_pre[i] = t;
    c_suf[i] = 30e-6 + m * kappa * D * 4.0 / 3e12 + m * 2e-8;
  }
  const std::vector<int> s_pre = assign(c_pre), s_suf = assign(c_suf);

  // ---- branches: projections and cascade levels before the full scans
  GV_HIP(hipEventRecord(fork, org));
  for (int j = 0; j < nside; ++j) GV_HIP(hipStreamWaitEvent(side[j], fork, 0));
  std::vector<ScoreArgs> last(ne);
  std::vector<Shape> last_sh(ne);
  for (int i = 0; i < ne; ++i) {
    hipStream_t st = side[s_pre[i]];
    BatchEntry& b = e[i];
    uint8_t* ws = b.ws;
    float* t = (float*)(ws + b.plan.off_t);
    float* qc = (float*)(ws + b.plan.off_qc);
    void* qhat = ws + b.plan.off_qhat;
    GV_TRY(project_impl(b.model, b.idx->fmt, b.Q, b.m, qc, t, qhat, st, b.plan.d_search, ws + b.plan.off_scan,
                        b.plan.region_bytes));
    GV_TRY(run_scan(b.idx, plans[i], ws + b.plan.off_scan, qhat, t, b.m, kappa, nullptr, nullptr, st, nullptr,
                    Part::Prefix, &last[i], &last_sh[i]));
  }
  for (int j = 0; j < nside; ++j) {
    GV_HIP(hipEventRecord(join[j], side[j]));
    GV_HIP(hipStreamWaitEvent(org, join[j], 0));
  }
  // ---- the full scans: one persistent queue launch per class, the classes on
  // the side streams (a class's workgroups take the CUs another class's
  // stragglers leave idle)
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, org, (int*)(qmem + off_heads), (int)cls.size());
  GV_HIP(hipGetLastError());
  GV_HIP(hipEventRecord(fork, org));
  for (int j = 0; j < nside; ++j) GV_HIP(hipStreamWaitEvent(side[j], fork, 0));
  // largest classes first, each onto the least loaded stream
  std::vector<double> c_cls(cls.size(), 0.0);
  for (size_t c = 0; c < cls.size(); ++c)
    for (int i : cls[c].members)
      c_cls[c] += (double)e[i].m * (double)e[i].idx->n_rows * (double)plans[i].dp;
  std::vector<int> corder(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) corder[c] = (int)c;
  std::sort(corder.begin(), corder.end(), [&](int x, int y) { return c_cls[x] > c_cls[y]; });
  std::vector<double> sload(nside, 0.0);
  for (int c : corder) {
    const int sj = (int)(std::min_element(sload.begin(), sload.end()) - sload.begin());
    sload[sj] += c_cls[c];
    std::vector<int64_t> offs(cls[c].members.size() + 1, 0);
    for (size_t j = 0; j < cls[c].members.size(); ++j) {
      const int i = cls[c].members[j];
      std::memcpy(upload->data() + off_args[c] + sizeof(ScoreArgs) * j, &last[i], sizeof(ScoreArgs));
      offs[j + 1] = offs[j] + last_sh[i].grid;
    }
    std::memcpy(upload->data() + off_off[c], offs.data(), sizeof(int64_t) * offs.size());
    const Shape& rep = last_sh[cls[c].members[0]];
    const int occ = scan_limits(cls[c].fmt, cls[c].dp, rep).occupancy;
    const int grid = (int)std::min<int64_t>(offs.back(), (int64_t)n_cu * occ);
    GV_TRY(dispatch_fmt_queue(cls[c].fmt, cls[c].dp, rep, grid, (const ScoreArgs*)(qmem + off_args[c]),
                              (const int64_t*)(qmem + off_off[c]), (int)cls[c].members.size(),
                              (int*)(qmem + off_heads) + c, side[sj]));
  }
  for (int j = 0; j < nside; ++j) {
    GV_HIP(hipEventRecord(join[j], side[j]));
    GV_HIP(hipStreamWaitEvent(org, join[j], 0));
  }
  // ---- branches: final selects and reranks
  GV_HIP(hipEventRecord(fork, org));
  for (int j = 0; j < nside; ++j) GV_HIP(hipStreamWaitEvent(side[j], fork, 0));
  for (int i = 0; i < ne; ++i) {
    hipStream_t st = side[s_suf[i]];
    BatchEntry& b = e[i];
    uint8_t* ws = b.ws;
    int32_t* cand = (int32_t*)(ws + b.plan.off_cand);
    float* csc = (float*)(ws + b.plan.off_csc);
    GV_TRY(run_scan(b.idx, plans[i], ws + b.plan.off_scan, ws + b.plan.off_qhat, (float*)(ws + b.plan.off_t), b.m,
                    kappa, cand, csc, st, nullptr, Part::Suffix));
    if (b.plan.stored) {
      float* qc = (float*)(ws + b.plan.off_qc);
      GV_TRY(rerank_stored_impl(b.idx, qc, b.m, cand, kappa, k, b.out_ids, b.out_scores, st));
    } else {
      GV_TRY(rerank_impl(b.idx, b.Q, b.m, cand, kappa, k, b.out_ids, b.out_scores, st, ws + b.plan.off_scan,
                         b.plan.region_bytes));
    }
  }
  for (int j = 0; j < nside; ++j) {
    GV_HIP(hipEventRecord(join[j], side[j]));
    GV_HIP(hipStreamWaitEvent(org, join[j], 0));
  }
  return GV_OK;
}

size_t batched_queue_bytes(int n_entries) {
  // at most one class per search: per class args, offsets and a head
  return (size_t)n_entries * (align256(sizeof(scan::ScoreArgs)) + align256(sizeof(int64_t) * 2) + 512) + 4096;
}

// ============================================================================ S4
namespace {

// One workgroup per query, sixteen wavefronts; each wavefront scores four
// candidate rows at a time so their loads are in flight together.
constexpr int kRerankThreads = 1024;

__device__ void sort_emit(double* s_score, int32_t* s_id, int64_t q, int kappa, int k, int32_t* __restrict__ out_ids,
                          float* __restrict__ out_scores);

// exact <q, x> of four candidate rows (a missing candidate, id outside [0, n),
// reads row 0 and is dropped by the caller) with FP64 accumulation of exact
// FP32 x FP32 products; each lane loads its part of the four rows with every
// load in flight before the first use (the rows are gathered: one memory
// latency per group of four).  Called by a whole wavefront; every lane gets
// the four sums.
__device__ inline void dot4(const float* __restrict__ X, int64_t n, int D, const float* __restrict__ qv,
                            const int32_t (&id)[4], bool vec, double (&acc)[4]) {
  const int lane = threadIdx.x & 63;
  const float* x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    x[u] = X + ((id[u] >= 0 && id[u] < n) ? (int64_t)id[u] : 0) * D;
    acc[u] = 0.0;
  }
  int j0 = 0;
  if (vec) {
    constexpr int kChunk = 4;  // float4 groups per lane per pass: 1024 coordinates of a row
    for (; j0 + 256 * kChunk <= D; j0 += 256 * kChunk) {
      float4 xv[4][kChunk], qq[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int j = j0 + 4 * (lane + 64 * c);
        qq[c] = *(const float4*)(qv + j);
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u][c] = *(const float4*)(x[u] + j);
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc[u] += (double)xv[u][c].x * (double)qq[c].x;
          acc[u] += (double)xv[u][c].y * (double)qq[c].y;
          acc[u] += (double)xv[u][c].z * (double)qq[c].z;
          acc[u] += (double)xv[u][c].w * (double)qq[c].w;
        }
    }
    for (int j = j0 + 4 * lane; j + 4 <= D; j += 256) {
      const float4 qq = *(const float4*)(qv + j);
      float4 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = *(const float4*)(x[u] + j);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[u] += (double)xv[u].x * (double)qq.x;
        acc[u] += (double)xv[u].y * (double)qq.y;
        acc[u] += (double)xv[u].z * (double)qq.z;
        acc[u] += (double)xv[u].w * (double)qq.w;
      }
    }
  } else {
    for (int j = lane; j < D; j += 64) {
      const double qj = (double)qv[j];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += (double)x[u][j] * qj;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    for (int o = 32; o > 0; o >>= 1) acc[u] += __shfl_xor(acc[u], o);
}

__device__ inline bool rerank_vec(const float* X, int D, const float* Q) {
  return (D % 4) == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)Q % 16) == 0;
}

__global__ __launch_bounds__(kRerankThreads) void k_rerank(const float* __restrict__ X, int64_t n, int D,
                                                           const float* __restrict__ Q,
                                                           const int32_t* __restrict__ cand, int kappa, int k,
                                                           int32_t* __restrict__ out_ids,
                                                           float* __restrict__ out_scores) {
  __shared__ double s_score[kMaxKappa];
  __shared__ int32_t s_id[kMaxKappa];
  constexpr int W = kRerankThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = blockIdx.x;
  const float* qv = Q + q * D;
  for (int i = tid; i < kMaxKappa; i += kRerankThreads) {
    s_score[i] = -INFINITY;
    s_id[i] = 0x7fffffff;
  }
  __syncthreads();
  const bool vec = rerank_vec(X, D, Q);
  for (int c0 = wave * 4; c0 < kappa; c0 += W * 4) {
    int32_t id[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) id[u] = (c0 + u < kappa) ? cand[q * kappa + c0 + u] : -1;
    double acc[4];
    dot4(X, n, D, qv, id, vec, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane == 0 && id[u] >= 0 && id[u] < n) {  // a missing candidate (non-finite query scores) is skipped
        s_score[c0 + u] = acc[u];
        s_id[c0 + u] = id[u];
      }
  }
  __syncthreads();
  sort_emit(s_score, s_id, q, kappa, k, out_ids, out_scores);
}

// Small batches: one workgroup per query leaves most of the device idle and
// takes one gathered-row latency per 64 candidates, so the scores are computed
// by many workgroups per query (kRerankPart candidates each, one round of
// loads) into FP64 scratch, and sorted by a second kernel.  Same arithmetic as
// k_rerank, same results.
constexpr int kRerankPart = 16;
constexpr int64_t kRerankSplitM = 256;
__global__ __launch_bounds__(256) void k_rerank_part(const float* __restrict__ X, int64_t n, int D,
                                                     const float* __restrict__ Q, const int32_t* __restrict__ cand,
                                                     int kappa, double* __restrict__ score) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = blockIdx.y;
  const int c0 = blockIdx.x * kRerankPart + wave * 4;
  if (c0 >= kappa) return;
  int32_t id[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) id[u] = (c0 + u < kappa) ? cand[q * kappa + c0 + u] : -1;
  double acc[4];
  dot4(X, n, D, Q + q * D, id, rerank_vec(X, D, Q), acc);
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (lane == 0 && c0 + u < kappa) score[q * kappa + c0 + u] = acc[u];
}

__global__ __launch_bounds__(kRerankThreads) void k_rerank_sort(int64_t n, const int32_t* __restrict__ cand, int kappa,
                                                                int k, const double* __restrict__ score,
                                                                int32_t* __restrict__ out_ids,
                                                                float* __restrict__ out_scores) {
  __shared__ double s_score[kMaxKappa];
  __shared__ int32_t s_id[kMaxKappa];
  const int64_t q = blockIdx.x;
  for (int i = threadIdx.x; i < kMaxKappa; i += kRerankThreads) {
    const int32_t id = i < kappa ? cand[q * kappa + i] : -1;
    const bool ok = id >= 0 && id < n;  // a missing candidate (non-finite query scores) is skipped
    s_score[i] = ok ? score[q * kappa + i] : -INFINITY;
    s_id[i] = ok ? id : 0x7fffffff;
  }
  __syncthreads();
  sort_emit(s_score, s_id, q, kappa, k, out_ids, out_scores);
}

// bitonic sort of the (score, id) pairs in LDS (score desc, then id asc) over
// the smallest power of two >= kappa slots (unused slots hold -inf), then the
// first k to the output row q; called by every thread of the workgroup
__device__ void sort_emit(double* s_score, int32_t* s_id, int64_t q, int kappa, int k, int32_t* __restrict__ out_ids,
                          float* __restrict__ out_scores) {
  const int tid = threadIdx.x;
  const int sn = pow2_at_least(kappa);
  for (int size = 2; size <= sn; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < sn; i += kRerankThreads) {
        const int j = i ^ stride;
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

// Rerank from the stored vectors (Section 3.3): <A_c q, x'> with x' = s_c x^
// over every stored coordinate, FP64 accumulation of exact products.  One
// workgroup per query; a wavefront scores one candidate at a time, each lane
// taking whole operand groups (EPL consecutive coordinates) of the candidate's
// row from its 32-row tile.
template <int FMT>
__global__ __launch_bounds__(kRerankThreads) void k_rerank_stored(
    const uint8_t* __restrict__ xlow, int dps, const float* __restrict__ scale, const uint8_t* __restrict__ tags,
    const int32_t* __restrict__ pos, int64_t n, int C, const float* __restrict__ qc,
    const int32_t* __restrict__ cand, int kappa, int k, int32_t* __restrict__ out_ids,
    float* __restrict__ out_scores) {
  __shared__ double s_score[kMaxKappa];
  __shared__ int32_t s_id[kMaxKappa];
  constexpr int W = kRerankThreads / 64;
  constexpr int EPL = FMT == GV_FP32 ? 1 : 8, KM = FMT == GV_FP32 ? 2 : 16;
  constexpr int EB = FMT == GV_FP32 ? 4 : (FMT == GV_FP8_E4M3 ? 1 : 2);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = blockIdx.x;
  for (int i = tid; i < kMaxKappa; i += kRerankThreads) {
    s_score[i] = -INFINITY;
    s_id[i] = 0x7fffffff;
  }
  __syncthreads();
  const int groups = dps / EPL;
  for (int r = wave; r < kappa; r += W) {
    const int32_t id = cand[q * kappa + r];
    if (id < 0 || id >= n) continue;  // a missing candidate is skipped
    const int c = tags[id];
    const int64_t p = pos[id];
    if (c >= C || p < 0) continue;    // a removed id has no stored vector
    const int64_t t = p / kTileRows;
    const int i = (int)(p - t * kTileRows);
    const float* qv = qc + (q * C + c) * (int64_t)dps;
    double acc = 0.0;
    for (int g = lane; g < groups; g += 64) {
      const int s = g * EPL / KM, half = (g * EPL % KM) / EPL;
      const int64_t off = ((t * (dps / KM) + s) * 64 + i + kTileRows * half) * EPL;  // in elements
      const uint8_t* src = xlow + off * EB;
      if constexpr (FMT == GV_FP32) {
        acc += (double)*(const float*)src * (double)qv[g];
      } else if constexpr (FMT == GV_FP8_E4M3) {
        const uint2 w = *(const uint2*)src;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          acc += from_fp8((uint8_t)(((e < 4 ? w.x : w.y) >> (8 * (e & 3))) & 255)) * (double)qv[g * 8 + e];
      } else {
        const uint4 w = *(const uint4*)src;
        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint16_t b = (uint16_t)((ww[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          acc += (FMT == GV_FP16 ? from_fp16(b) : from_bf16(b)) * (double)qv[g * 8 + e];
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
      s_score[r] = acc * (double)scale[c];  // exact: s_c is a power of two
      s_id[r] = id;
    }
  }
  __syncthreads();
  sort_emit(s_score, s_id, q, kappa, k, out_ids, out_scores);
}

}  // namespace

gv_status rerank_stored_impl(const gv_index* idx, const float* qc, int64_t m, const int32_t* cand, int kappa, int k,
                             int32_t* out_ids, float* out_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  const dim3 g((unsigned)m), b(kRerankThreads);
  const uint8_t* xl = (const uint8_t*)idx->xlow;
  switch (idx->fmt) {
    case GV_FP32: hipLaunchKernelGGL(k_rerank_stored<GV_FP32>, g, b, 0, st, xl, idx->dp, idx->scale, idx->tags, idx->pos, idx->n, idx->C, qc, cand, kappa, k, out_ids, out_scores); break;
    case GV_FP16: hipLaunchKernelGGL(k_rerank_stored<GV_FP16>, g, b, 0, st, xl, idx->dp, idx->scale, idx->tags, idx->pos, idx->n, idx->C, qc, cand, kappa, k, out_ids, out_scores); break;
    case GV_BF16: hipLaunchKernelGGL(k_rerank_stored<GV_BF16>, g, b, 0, st, xl, idx->dp, idx->scale, idx->tags, idx->pos, idx->n, idx->C, qc, cand, kappa, k, out_ids, out_scores); break;
    default: hipLaunchKernelGGL(k_rerank_stored<GV_FP8_E4M3>, g, b, 0, st, xl, idx->dp, idx->scale, idx->tags, idx->pos, idx->n, idx->C, qc, cand, kappa, k, out_ids, out_scores); break;
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
}

gv_status rerank_impl(const gv_index* idx, const float* Q, int64_t m, const int32_t* cand, int kappa, int k,
                      int32_t* out_ids, float* out_scores, hipStream_t st, void* scratch, size_t scratch_bytes) {
  if (m == 0) return GV_OK;
  if (scratch && m <= kRerankSplitM && scratch_bytes >= sizeof(double) * (size_t)m * kappa) {
    double* score = (double*)scratch;
    hipLaunchKernelGGL(k_rerank_part, dim3((unsigned)((kappa + kRerankPart - 1) / kRerankPart), (unsigned)m),
                       dim3(256), 0, st, idx->X, idx->n, idx->D, Q, cand, kappa, score);
    hipLaunchKernelGGL(k_rerank_sort, dim3((unsigned)m), dim3(kRerankThreads), 0, st, idx->n, cand, kappa, k, score,
                       out_ids, out_scores);
  } else {
    hipLaunchKernelGGL(k_rerank, dim3((unsigned)m), dim3(kRerankThreads), 0, st, idx->X, idx->n, idx->D, Q, cand,
                       kappa, k, out_ids, out_scores);
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace gv
