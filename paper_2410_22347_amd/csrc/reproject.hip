// Re-projection of stored vectors for streaming search (Section 3, streaming
// vector search): an index that stores the full-dimension coordinates
// y = P_c W x (flexible storage at d = D, Section 3.3, with no copy of X) is
// carried over to refitted projections without X.  Per cluster,
//   y' = P'_c W' (P_c W)^-1 y = B'_c A_c^T y,
// since (P_c W)^-1 = W^-1 P_c^T = (P_c W+)^T = A_c^T when P_c is orthogonal
// (d = D) and K_Q has full rank.  Vectors inserted since are encoded with the
// new projections, y' = B'_c x; removed ones are dropped.  The landmarks stay,
// so every kept vector keeps its cluster.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

// dense FP32 copy of the stored vectors: Y[p][j] = s_c x^[p][j] (exact), for
// stored rows p (padding rows become zero)
template <int FMT>
__global__ void k_dequant_rows(const uint8_t* __restrict__ xlow, int dp, int64_t n_pad, const int64_t* __restrict__ off,
                               int C, const float* __restrict__ scale, const int32_t* __restrict__ ids, int d,
                               float* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pad * d) return;
  const int64_t p = e / d;
  const int j = (int)(e - p * d);
  int lo = 0, hi = C - 1;  // cluster of stored row p: last c with off[c] <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  if (ids[p] < 0) {
    Y[e] = 0.0f;
    return;
  }
  constexpr int KM = FMT == GV_FP32 ? 2 : 16, EPL = FMT == GV_FP32 ? 1 : 8;
  const int64_t o = tiled_offset(p, j, dp, KM, EPL);
  double x;
  if (FMT == GV_FP32) x = (double)((const float*)xlow)[o];
  else if (FMT == GV_FP16) x = from_fp16(((const uint16_t*)xlow)[o]);
  else if (FMT == GV_BF16) x = from_bf16(((const uint16_t*)xlow)[o]);
  else x = from_fp8(xlow[o]);
  Y[e] = (float)(x * (double)scale[lo]);  // exact: a stored value times a power of two
}

// removed ids leave the id space's clusters
__global__ void k_drop_removed(uint8_t* __restrict__ tags, const uint8_t* __restrict__ keep, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !keep[i]) tags[i] = 255;
}

// gather lists of the new grouping: stored row p of the new index takes old
// stored row pos_old[id] (ids below n_old) or inserted row id - n_old
__global__ void k_split_sources(const int64_t* __restrict__ ids64, int64_t n_pad, int64_t n_old,
                                const int32_t* __restrict__ pos_old, int64_t* __restrict__ src) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pad) return;
  const int64_t id = ids64[p];
  src[p] = id < 0 ? 0 : (id < n_old ? (int64_t)pos_old[id] : id - n_old);
}

template <int FMT>
gv_status dequant(const gv_index* in, float* Y, hipStream_t st) {
  const int64_t total = in->n_pad * in->d;
  hipLaunchKernelGGL(k_dequant_rows<FMT>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     (const uint8_t*)in->xlow, in->dp, in->n_pad, in->offsets, in->C, in->scale, in->ids, in->d, Y);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace

gv_status reproject_impl(const gv_model* m0, const gv_model* m1, const gv_index* in, const uint8_t* keep,
                         const float* X_new, int64_t n_new, int fmt, hipStream_t st, gv_index* out) {
  const int C = m1->C, D = m1->D, d = D;
  const int64_t n_old = in->n, n = n_old + n_new;
  const size_t DD = (size_t)D * D;

  // ------------------------------------------------ tags of the id space
  GV_HIP(hipMemcpyAsync(out->tags, in->tags, n_old, hipMemcpyDeviceToDevice, st));
  if (keep)
    hipLaunchKernelGGL(k_drop_removed, dim3((unsigned)((n_old + 255) / 256)), dim3(256), 0, st, out->tags, keep, n_old);
  if (n_new > 0) GV_TRY(tags_impl(m1, X_new, n_new, out->tags + n_old, st));
  GV_HIP(hipGetLastError());

  // ------------------------------------------------ grouping (old rows first in each segment: smaller ids)
  TempBuf<int64_t> ibuf(st);
  GV_TRY(group_rows(n, C, out->dp, fmt, st, out, &ibuf.p));
  const int64_t* ids64 = ibuf.p;
  std::vector<uint8_t> h_tags(n);
  GV_HIP(hipMemcpyAsync(h_tags.data(), out->tags, n, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> old_cnt(C, 0);
  for (int64_t i = 0; i < n_old; ++i)
    if (h_tags[i] < C) ++old_cnt[h_tags[i]];

  // ------------------------------------------------ T_c = B'_c A_c^T (D x D per cluster, FP64)
  TempBuf<double> tbuf(st);
  TempBuf<float> ybuf(st), vbuf(st);
  TempBuf<int64_t> sbuf(st);
  GV_HIP(tbuf.alloc(sizeof(double) * DD * C));
  GV_HIP(ybuf.alloc(sizeof(float) * std::max<int64_t>(in->n_pad, 1) * d));
  GV_HIP(vbuf.alloc(sizeof(float) * std::max<int64_t>(out->n_pad, 1) * d));
  GV_HIP(sbuf.alloc(sizeof(int64_t) * std::max<int64_t>(out->n_pad, 1)));
  double* T = tbuf.p;
  float* Y = ybuf.p;
  float* v = vbuf.p;
  int64_t* src = sbuf.p;
  GV_HIP(hipMemsetAsync(v, 0, sizeof(float) * out->n_pad * d, st));
  {
    GemmOperand<double> b1{m1->B, D, nullptr, Layout::RowMajor, (int64_t)DD};
    GemmOperand<double> a0{m0->A, D, nullptr, Layout::RowMajor, (int64_t)DD};
    GemmOut to{T, D, 0, 0, nullptr, (int64_t)DD};
    GV_TRY(gemm_f64<double, double>(D, D, D, b1, a0, Epi::StoreF64, to, st, C));
  }
  // ------------------------------------------------ stored values s_c x^ as dense FP32 rows
  switch (in->fmt) {
    case GV_FP32: GV_TRY(dequant<GV_FP32>(in, Y, st)); break;
    case GV_FP16: GV_TRY(dequant<GV_FP16>(in, Y, st)); break;
    case GV_BF16: GV_TRY(dequant<GV_BF16>(in, Y, st)); break;
    default: GV_TRY(dequant<GV_FP8_E4M3>(in, Y, st)); break;
  }
  hipLaunchKernelGGL(k_split_sources, dim3((unsigned)((out->n_pad + 255) / 256)), dim3(256), 0, st, ids64, out->n_pad,
                     n_old, in->pos, src);
  GV_HIP(hipGetLastError());
  // ------------------------------------------------ y' = fl32(T_c y) for kept rows, fl32(B'_c x) for inserted ones
  for (int c = 0; c < C; ++c) {
    const int64_t a = out->h_offsets[c], co = old_cnt[c], cn = out->h_counts[c] - old_cnt[c];
    if (co > 0) {
      GemmOperand<float> yo{Y, d, src + a, Layout::RowMajor};
      GemmOperand<double> to{T + DD * c, D, nullptr, Layout::RowMajor};
      GV_TRY(gemm_f64<float, double>(co, d, D, yo, to, Epi::StoreF32, GemmOut{v + a * d, d, 0, 0, nullptr}, st));
    }
    if (cn > 0) {
      GemmOperand<float> xo{X_new, D, src + a + co, Layout::RowMajor};
      GemmOperand<double> bo{m1->B + (int64_t)c * d * D, D, nullptr, Layout::RowMajor};
      GV_TRY(gemm_f64<float, double>(cn, d, D, xo, bo, Epi::StoreF32, GemmOut{v + (a + co) * d, d, 0, 0, nullptr},
                                     st));
    }
  }
  // ------------------------------------------------ per-cluster scale and storage
  GV_TRY(quantize_rows(v, d, fmt, st, out));
  GV_HIP(hipStreamSynchronize(st));
  return GV_OK;
}

}  // namespace gv
