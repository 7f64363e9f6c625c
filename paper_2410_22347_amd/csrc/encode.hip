// Index build (Section 4 of the paper): cluster tags (Eq. 9) and reduced
// vectors x_low = B_c x (Eq. 10), grouped by cluster.
//
// Layout in HBM (all device memory owned by the index):
//   tags[n]            uint8, cluster of each original row;
//   offsets[C+1]       int64, start of each cluster's stored segment; segments
//                      are padded to a multiple of 32 rows (one tile);
//   seg_end[C]         int64, first padding row of each segment;
//   ids[n_pad]         int32, original row id of each stored row (stable:
//                      increasing inside a segment), -1 for padding rows;
//   xlow[n_pad][d_pad] storage format, zero padded, in matrix-core operand
//                      tiles (see tiled_offset): one k-step of a 32-row tile is
//                      one contiguous block that a wavefront loads in one go;
//   scale[C]           FP32 power-of-two s_c; the stored value is rnd(v / s_c);
//   X[n][D]            FP32 original vectors for the rerank (copied or borrowed).
// The grouped layout replaces the paper's interleaved (tag, x_low) pairs: a
// scan reads each cluster's segment contiguously and needs one query view per
// segment instead of one tag lookup per vector.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

constexpr int kBlockRows = 1024;

__global__ void k_argmax_u8(const double* __restrict__ dots, int64_t rows, int C, uint8_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double* d = dots + r * C;
  int best = 0;
  double bv = d[0];
  for (int c = 1; c < C; ++c)
    if (d[c] > bv) {
      bv = d[c];
      best = c;
    }
  out[r] = (uint8_t)best;
}

// per-block cluster histogram: hist[b * C + c]
__global__ void k_block_hist(const uint8_t* __restrict__ tags, int64_t n, int C, int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  for (int c = threadIdx.x; c < C; c += blockDim.x) h[c] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * kBlockRows;
  for (int i = threadIdx.x; i < kBlockRows; i += blockDim.x) {
    int64_t r = r0 + i;
    if (r < n && tags[r] < C) atomicAdd(&h[tags[r]], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) hist[(int64_t)blockIdx.x * C + c] = h[c];
}

// stable scatter: rows of block b are placed in increasing id order after base[c][b]
__global__ void k_block_scatter(const uint8_t* __restrict__ tags, int64_t n, int C, const int64_t* __restrict__ base,
                                int64_t nblocks, int32_t* __restrict__ ids, int64_t* __restrict__ ids64,
                                int32_t* __restrict__ pos) {
  __shared__ uint8_t t[kBlockRows];
  __shared__ int64_t cnt[256];
  const int64_t r0 = (int64_t)blockIdx.x * kBlockRows;
  for (int i = threadIdx.x; i < kBlockRows; i += blockDim.x) t[i] = (r0 + i < n) ? tags[r0 + i] : 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) cnt[c] = base[(int64_t)c * nblocks + blockIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int rows = (int)min<int64_t>(kBlockRows, n - r0);
    for (int i = 0; i < rows; ++i) {
      if (t[i] >= C) {  // an absent id (removed vector): no stored row
        pos[r0 + i] = -1;
        continue;
      }
      int64_t p = cnt[t[i]]++;
      ids[p] = (int32_t)(r0 + i);
      ids64[p] = r0 + i;
      pos[r0 + i] = (int32_t)p;
    }
  }
}

// per-cluster max |v| (non-negative floats order like their bit patterns)
__global__ void k_segment_amax(const float* __restrict__ v, int d, const int64_t* __restrict__ off,
                               uint32_t* __restrict__ amax_bits) {
  const int c = blockIdx.y;
  const int64_t a = off[c] * d, b = off[c + 1] * d;
  uint32_t m = 0;
  for (int64_t e = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < b; e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t u = __float_as_uint(fabsf(v[e]));
    m = max(m, u);
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&amax_bits[c], m);
}

template <int FMT>
__global__ void k_quantize(const float* __restrict__ v, int64_t n_pad, int d, int dp, const int64_t* __restrict__ off,
                           int C, const float* __restrict__ scale, const int32_t* __restrict__ ids,
                           void* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pad * dp) return;
  const int64_t p = e / dp;
  const int j = (int)(e - p * dp);
  // cluster of stored row p: last c with off[c] <= p
  int lo = 0, hi = C - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const float x = (j < d && ids[p] >= 0) ? v[p * d + j] : 0.0f;
  const double y = (double)x / (double)scale[lo];  // exact: scale is a power of two
  const int64_t o = tiled_offset(p, j, dp, FMT == GV_FP32 ? 2 : 16, FMT == GV_FP32 ? 1 : 8);
  if (FMT == GV_FP32) {
    ((float*)out)[o] = x;
  } else if (FMT == GV_FP16) {
    ((uint16_t*)out)[o] = to_fp16(y);
  } else if (FMT == GV_BF16) {
    ((uint16_t*)out)[o] = to_bf16(y);
  } else {
    ((uint8_t*)out)[o] = to_fp8(y);
  }
}

}  // namespace

// tag_i = arg-max_c <x_i, mu_c> in FP64, lowest c on ties (the cluster-tag
// equation of Section 4)
gv_status tags_impl(const gv_model* model, const float* X, int64_t n, uint8_t* tags, hipStream_t st) {
  const int C = model->C, D = model->D;
  const int64_t chunk = std::min<int64_t>(n, 1 << 20);
  TempBuf<double> dbuf(st);
  GV_HIP(dbuf.alloc(sizeof(double) * chunk * C));
  double* dots = dbuf.p;
  gv_status s = GV_OK;
  for (int64_t s0 = 0; s0 < n && s == GV_OK; s0 += chunk) {
    const int64_t rows = std::min(chunk, n - s0);
    GemmOperand<float> xo{X + s0 * D, D, nullptr, Layout::RowMajor};
    GemmOperand<double> mo{model->mu, D, nullptr, Layout::RowMajor};
    s = gemm_f64<float, double>(rows, C, D, xo, mo, Epi::StoreF64, GemmOut{dots, C, 0, 0, nullptr}, st);
    if (s == GV_OK)
      hipLaunchKernelGGL(k_argmax_u8, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, dots, rows, C,
                         tags + s0);
  }
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

// Groups the rows 0..n-1 of idx->tags by tag (stable, increasing ids inside a
// cluster; tags >= C are absent rows), pads every segment to whole tiles, and
// allocates and fills offsets, seg_end, ids, pos and the storage xlow of the
// index (dp padded columns of format fmt).  *ids64: device n_pad original ids
// of the stored rows (-1 padding), to be freed by the caller with hipFreeAsync.
gv_status group_rows(int64_t n, int C, int dp, int fmt, hipStream_t st, gv_index* idx, int64_t** ids64_out) {
  const int64_t nb = (n + kBlockRows - 1) / kBlockRows;
  TempBuf<int32_t> hbuf(st);
  TempBuf<int64_t> bbuf(st), ibuf(st);
  GV_HIP(hbuf.alloc(sizeof(int32_t) * nb * C));
  GV_HIP(bbuf.alloc(sizeof(int64_t) * nb * C));
  int32_t* hist = hbuf.p;
  int64_t* base = bbuf.p;
  hipLaunchKernelGGL(k_block_hist, dim3((unsigned)nb), dim3(256), 0, st, idx->tags, n, C, hist);
  GV_HIP(hipGetLastError());
  std::vector<int32_t> h_hist((size_t)nb * C);
  GV_HIP(hipMemcpyAsync(h_hist.data(), hist, sizeof(int32_t) * nb * C, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> h_base((size_t)nb * C);
  idx->h_offsets.assign(C + 1, 0);
  idx->h_counts.assign(C, 0);
  int64_t run = 0, rows = 0;
  for (int c = 0; c < C; ++c) {
    idx->h_offsets[c] = run;
    int64_t cnt = 0;
    for (int64_t b = 0; b < nb; ++b) {
      h_base[(size_t)c * nb + b] = run + cnt;
      cnt += h_hist[(size_t)b * C + c];
    }
    idx->h_counts[c] = cnt;
    rows += cnt;
    run += (cnt + kTileRows - 1) / kTileRows * kTileRows;
  }
  idx->h_offsets[C] = run;
  idx->n_pad = run;
  idx->n_rows = rows;
  GV_HIP(dev_malloc((void**)&idx->ids, sizeof(int32_t) * std::max<int64_t>(run, 1)));
  GV_HIP(dev_malloc((void**)&idx->pos, sizeof(int32_t) * std::max<int64_t>(n, 1)));
  GV_HIP(dev_malloc(&idx->xlow, (size_t)std::max<int64_t>(run, 1) * dp * fmt_bytes(fmt)));
  GV_HIP(ibuf.alloc(sizeof(int64_t) * std::max<int64_t>(run, 1)));
  int64_t* ids64 = ibuf.p;
  GV_HIP(hipMemsetAsync(idx->ids, 0xFF, sizeof(int32_t) * run, st));   // -1: padding
  GV_HIP(hipMemsetAsync(ids64, 0xFF, sizeof(int64_t) * run, st));
  GV_HIP(hipMemcpyAsync(base, h_base.data(), sizeof(int64_t) * nb * C, hipMemcpyHostToDevice, st));
  GV_HIP(hipMemcpyAsync(idx->offsets, idx->h_offsets.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, st));
  std::vector<int64_t> h_end(C);
  for (int c = 0; c < C; ++c) h_end[c] = idx->h_offsets[c] + idx->h_counts[c];
  GV_HIP(hipMemcpyAsync(idx->seg_end, h_end.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_block_scatter, dim3((unsigned)nb), dim3(64), 0, st, idx->tags, n, C, base, nb, idx->ids, ids64,
                     idx->pos);
  GV_HIP(hipGetLastError());
  GV_HIP(hipStreamSynchronize(st));  // the host staging vectors end with this block
  *ids64_out = ibuf.release();
  return GV_OK;
}

// Per-cluster power-of-two scale from the amax of the grouped FP32 rows v
// (n_pad x d, padding rows zero) and the rounded storage of every row.
gv_status quantize_rows(const float* v, int d, int fmt, hipStream_t st, gv_index* idx) {
  const int C = idx->C, dp = idx->dp;
  const int64_t n_pad = idx->n_pad;
  TempBuf<uint32_t> abuf(st);
  GV_HIP(abuf.alloc(sizeof(uint32_t) * C));
  uint32_t* amax = abuf.p;
  GV_HIP(hipMemsetAsync(amax, 0, sizeof(uint32_t) * C, st));
  hipLaunchKernelGGL(k_segment_amax, dim3(64, C), dim3(256), 0, st, v, d, idx->offsets, amax);
  GV_HIP(hipGetLastError());
  std::vector<uint32_t> h_amax(C);
  GV_HIP(hipMemcpyAsync(h_amax.data(), amax, sizeof(uint32_t) * C, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  std::vector<float> h_scale(C);
  for (int c = 0; c < C; ++c) {
    float a;
    std::memcpy(&a, &h_amax[c], 4);
    h_scale[c] = pow2_scale(a, scale_target(fmt));
  }
  GV_HIP(hipMemcpyAsync(idx->scale, h_scale.data(), sizeof(float) * C, hipMemcpyHostToDevice, st));
  const int64_t total = n_pad * dp;
  const unsigned grid = (unsigned)((total + 255) / 256);
  switch (fmt) {
    case GV_FP32:
      hipLaunchKernelGGL(k_quantize<GV_FP32>, dim3(grid), dim3(256), 0, st, v, n_pad, d, dp, idx->offsets, C,
                         idx->scale, idx->ids, idx->xlow);
      break;
    case GV_FP16:
      hipLaunchKernelGGL(k_quantize<GV_FP16>, dim3(grid), dim3(256), 0, st, v, n_pad, d, dp, idx->offsets, C,
                         idx->scale, idx->ids, idx->xlow);
      break;
    case GV_BF16:
      hipLaunchKernelGGL(k_quantize<GV_BF16>, dim3(grid), dim3(256), 0, st, v, n_pad, d, dp, idx->offsets, C,
                         idx->scale, idx->ids, idx->xlow);
      break;
    default:
      hipLaunchKernelGGL(k_quantize<GV_FP8_E4M3>, dim3(grid), dim3(256), 0, st, v, n_pad, d, dp, idx->offsets, C,
                         idx->scale, idx->ids, idx->xlow);
      break;
  }
  GV_HIP(hipGetLastError());
  GV_HIP(hipStreamSynchronize(st));
  return GV_OK;
}

gv_status encode_impl(const gv_model* model, const float* X, int64_t n, int fmt, hipStream_t st, gv_index* idx) {
  const int C = model->C, d = model->d, D = model->D, dp = pad_dim(d);

  // ------------------------------------------------ tags, FP64 arg-max (Eq. 9)
  GV_TRY(tags_impl(model, X, n, idx->tags, st));

  // ------------------------------------------------ stable grouping by tag, padded segments
  TempBuf<int64_t> ibuf(st);
  GV_TRY(group_rows(n, C, dp, fmt, st, idx, &ibuf.p));
  const int64_t* ids64 = ibuf.p;
  const int64_t n_pad = idx->n_pad;

  // ------------------------------------------------ x_low = fl32(B_c x), FP64 accumulation (Eq. 10)
  TempBuf<float> vbuf(st);
  GV_HIP(vbuf.alloc(sizeof(float) * std::max<int64_t>(n_pad, 1) * d));
  float* v = vbuf.p;
  GV_HIP(hipMemsetAsync(v, 0, sizeof(float) * n_pad * d, st));
  for (int c = 0; c < C; ++c) {
    const int64_t a = idx->h_offsets[c], nc = idx->h_counts[c];
    if (nc == 0) continue;
    GemmOperand<float> xo{X, D, ids64 + a, Layout::RowMajor};
    GemmOperand<double> bo{model->B + (int64_t)c * d * D, D, nullptr, Layout::RowMajor};
    GV_TRY(gemm_f64<float, double>(nc, d, D, xo, bo, Epi::StoreF32, GemmOut{v + a * d, d, 0, 0, nullptr}, st));
  }

  // ------------------------------------------------ per-cluster scale and quantisation
  GV_TRY(quantize_rows(v, d, fmt, st, idx));
  GV_HIP(hipStreamSynchronize(st));
  return GV_OK;
}

}  // namespace gv
