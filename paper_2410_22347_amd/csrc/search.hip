// Search path on gfx950: eager views (S1), grouped reduced scoring (S2) fused
// with a per-query top-kappa filter (S3), merge of the partial lists, and the
// full-dimension rerank (S4).  Algorithm 1 of the paper with the eager inner
// product of Algorithm 4 and an exhaustive main step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "search_common.hpp"

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

}  // namespace

gv_status project_impl(const gv_model* model, int fmt, const float* Q, int64_t m, float* qc, float* t, void* qhat,
                       hipStream_t st) {
  const int C = model->C, d = model->d, D = model->D, dp = pad16(d);
  float* tmp = nullptr;
  if (!qc) {
    GV_HIP(hipMallocAsync((void**)&tmp, sizeof(float) * m * C * dp, st));
    qc = tmp;
  }
  // q_c = fl32(A_c q), FP64 accumulation; columns j of the stacked A map to (c, j % d)
  GemmOperand<float> qo{Q, D, nullptr, Layout::RowMajor};
  GemmOperand<double> ao{model->A, D, nullptr, Layout::RowMajor};
  gv_status s = gemm_f64<float, double>(m, (int64_t)C * d, D, qo, ao, Epi::StoreF32Proj,
                                        GemmOut{qc, (int64_t)C * dp, d, dp, nullptr}, st);
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

// ============================================================================ S2 + S3
//
// One workgroup owns a block of queries and a contiguous range ("split") of
// row tiles; tiles never straddle two clusters, so a tile meets one eager view
// q_c per query, held in registers as the matrix-core B operand.  Scores leave
// the accumulators only through a threshold filter: a score below the query's
// current threshold tau can never enter the top kappa, so only survivors are
// written, as 64-bit keys (score desc, id asc), to a per-(query, split) buffer
// of kCap slots.  A buffer close to full is compacted to its kappa best keys and
// tau is raised to the kappa-th score.  At the end each buffer keeps at most
// kappa keys; a tree of merge launches reduces the lists to the final kappa.
//
// Threshold cascade: a scan over every s-th tile (a uniform sample of the
// grouped rows) yields, per query, the kappa-th best score of the sample -- a
// valid lower bound of the kappa-th best score of the whole database.  Seeding
// the next, denser scan with it keeps the survivors near kappa * s per query
// instead of kappa * ln(rows) per split.  The last scan covers every tile.
namespace {

constexpr int kCap = 2048;  // candidate slots per (query, split)

struct ScoreArgs {
  const uint8_t* xlow;    // n x dp, storage format
  const int32_t* ids;     // grouped position -> original id
  const float* scale;     // C
  const int64_t* offsets; // C + 1
  const uint8_t* qhat;    // m x C x dp, storage format
  const float* qscale;    // m x C
  const float* tau_init;  // m seed thresholds, or null (-inf)
  uint64_t* buf;          // m x P x kCap keys
  int32_t* cnt_out;       // m x P
  int64_t m;
  int C, dp, ks, kappa, P, nqb;
  int stride;             // scan every stride-th tile
  int xcd_map;            // 1: splits are pinned to XCDs (needs P % 8 == 0)
};

template <int FMT, int KSM, int NB, bool SHARED>
__global__ __launch_bounds__(256, 1) void k_score_select(ScoreArgs a) {
  using Op = MfmaOp<FMT>;
  using S = typename Op::S;
  using T = typename Op::T;
  constexpr int QWG = SHARED ? 32 * NB : 4 * 32 * NB;   // queries per workgroup
  constexpr int RPI = SHARED ? 128 : 32;                // rows per tile
  constexpr int LIMIT = kCap - RPI;                     // compact above this

  __shared__ int64_t s_off[257];
  __shared__ int32_t s_tpre[257];
  __shared__ int32_t s_cnt[QWG];
  __shared__ float s_tau[QWG];
  __shared__ int32_t s_list[QWG];
  __shared__ int32_t s_nlist;
  __shared__ uint64_t s_stage[256];
  __shared__ uint32_t s_kept;
  __shared__ SelectSmem sel;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int C = a.C;

  // ---- workgroup -> (query block, split); splits pinned to one XCD when asked
  int qb, p;
  if (a.xcd_map) {
    const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
    qb = j % a.nqb;
    p = (j / a.nqb) * 8 + x;
  } else {
    qb = blockIdx.x % a.nqb;
    p = blockIdx.x / a.nqb;
  }
  const int64_t q0 = (int64_t)qb * QWG;
  const int64_t wq0 = SHARED ? q0 : q0 + wave * 32 * NB;

  for (int c = tid; c <= C; c += 256) s_off[c] = a.offsets[c];
  for (int i = tid; i < QWG; i += 256) {
    const int64_t q = q0 + i;
    s_cnt[i] = 0;
    s_tau[i] = (q < a.m) ? (a.tau_init ? a.tau_init[q] : -INFINITY) : INFINITY;
  }
  __syncthreads();
  if (tid == 0) {
    s_tpre[0] = 0;
    for (int c = 0; c < C; ++c) s_tpre[c + 1] = s_tpre[c] + (int32_t)((s_off[c + 1] - s_off[c] + RPI - 1) / RPI);
  }
  __syncthreads();
  const int64_t ntiles = s_tpre[C];
  const int64_t nvirt = (ntiles + a.stride - 1) / a.stride;
  const int64_t v_begin = nvirt * p / a.P, v_end = nvirt * (p + 1) / a.P;

  const int half = lane >> 5, col = lane & 31;
  const int64_t kofs = (int64_t)(half * Op::EPL) * Op::EB;  // this lane's byte offset in a k-step
  T bq[NB][KSM];
  float st[NB];      // s_c * t_{q,c} for this lane's queries (times the operand widening)
  float tau_s[NB];   // thresholds in the accumulator domain
  int cur_c = -1;

  auto locate = [&](int64_t v, int& c, int64_t& row0, int64_t& row_end) {
    const int64_t tile = v * a.stride;
    int lo = 0, hi = C - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (s_tpre[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    c = lo;
    row0 = s_off[c] + (tile - s_tpre[c]) * RPI;
    row_end = s_off[c + 1];
  };
  auto load_rows = [&](S (&dst)[KSM], int64_t row0, int64_t row_end) {
    const int64_t base = row0 + (SHARED ? wave * 32 : 0);
    const int64_t r = base + col;
    const int64_t rr = r < row_end ? r : (base < row_end ? base : row0);
    const uint8_t* rp = a.xlow + rr * (int64_t)a.dp * Op::EB + kofs;
#pragma unroll
    for (int s = 0; s < KSM; ++s)
      if (s < a.ks) dst[s] = *(const S*)(rp + (int64_t)(s * Op::KM) * Op::EB);
  };
  auto refresh_tau = [&]() {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int lq = (int)(wq0 - q0) + nb * 32 + col;
      tau_s[nb] = s_tau[lq] / st[nb];
    }
  };

  S cur[KSM], nxt[KSM];
  int c_cur = 0;
  int64_t r0_cur = 0, re_cur = 0;
  if (v_begin < v_end) {
    locate(v_begin, c_cur, r0_cur, re_cur);
    load_rows(cur, r0_cur, re_cur);
  }

  for (int64_t v = v_begin; v < v_end; ++v) {
    // prefetch the next tile's rows while this one is scored
    int c_nxt = 0;
    int64_t r0_nxt = 0, re_nxt = 0;
    if (v + 1 < v_end) {
      locate(v + 1, c_nxt, r0_nxt, re_nxt);
      load_rows(nxt, r0_nxt, re_nxt);
    }
    const int c = c_cur;
    const int64_t row_end = re_cur;

    if (c != cur_c) {
      cur_c = c;
      const float sc = a.scale[c] * (Op::kScale * Op::kScale > 0.0f ? 1.0f / (Op::kScale * Op::kScale) : 1.0f);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t q = wq0 + nb * 32 + col;
        const bool qv = q < a.m;
        const uint8_t* qp = a.qhat + ((qv ? q : 0) * C + c) * (int64_t)a.dp * Op::EB + kofs;
#pragma unroll
        for (int s = 0; s < KSM; ++s) {
          if (s < a.ks && qv) bq[nb][s] = Op::cvt(*(const S*)(qp + (int64_t)(s * Op::KM) * Op::EB));
          else bq[nb][s] = zero_op<T>();
        }
        st[nb] = sc * (qv ? a.qscale[q * C + c] : 1.0f);
      }
      refresh_tau();
    }

    const int64_t base = r0_cur + (SHARED ? wave * 32 : 0);
    if (base < row_end) {
      f32x16 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x16{0};
#pragma unroll
      for (int s = 0; s < KSM; ++s) {
        if (s < a.ks) {
          const T av = Op::cvt(cur[s]);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = Op::mma(av, bq[nb][s], acc[nb]);
        }
      }
      // epilogue: lane holds query col, rows base + (i%4) + 8*(i/4) + 4*half
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float mx = -INFINITY;
#pragma unroll
        for (int i = 0; i < 16; ++i) mx = fmaxf(mx, acc[nb][i]);
        if (mx >= tau_s[nb]) {
          const int lq = (int)(wq0 - q0) + nb * 32 + col;
          const int64_t q = q0 + lq;
          uint64_t* qbuf = a.buf + ((q * a.P) + p) * (int64_t)kCap;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int64_t row = base + (i & 3) + 8 * (i >> 2) + 4 * half;
            if (row < row_end && acc[nb][i] >= tau_s[nb]) {
              const float score = acc[nb][i] * st[nb];
              const uint32_t id = (uint32_t)a.ids[row];
              const int slot = atomicAdd(&s_cnt[lq], 1);
              qbuf[slot] = make_key(score, id);
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- compaction of the queries whose buffers are nearly full
    if (tid == 0) s_nlist = 0;
    __syncthreads();
    for (int i = tid; i < QWG; i += 256)
      if (s_cnt[i] > LIMIT) s_list[atomicAdd(&s_nlist, 1)] = i;
    __syncthreads();
    const int nlist = s_nlist;
    for (int li = 0; li < nlist; ++li) {
      const int lq = s_list[li];
      uint64_t* qbuf = a.buf + (((q0 + lq) * a.P) + p) * (int64_t)kCap;
      const int cnt = s_cnt[lq];
      const uint64_t kth = block_kth(qbuf, cnt, a.kappa, sel);
      if (tid == 0) s_kept = 0;
      __syncthreads();
      for (int i = tid; i < cnt; i += 256) {
        uint64_t k = qbuf[i];
        if (k >= kth) s_stage[atomicAdd(&s_kept, 1u)] = k;
      }
      __syncthreads();
      for (int i = tid; i < a.kappa; i += 256) qbuf[i] = s_stage[i];
      if (tid == 0) {
        s_cnt[lq] = a.kappa;
        s_tau[lq] = fmaxf(s_tau[lq], key_score(kth));
      }
      __syncthreads();
    }
    if (nlist > 0) refresh_tau();

#pragma unroll
    for (int s = 0; s < KSM; ++s) cur[s] = nxt[s];
    c_cur = c_nxt;
    r0_cur = r0_nxt;
    re_cur = re_nxt;
  }

  // ---- final: keep at most kappa keys per (query, split)
  __syncthreads();
  for (int lq = 0; lq < QWG; ++lq) {
    const int64_t q = q0 + lq;
    if (q >= a.m) break;
    uint64_t* qbuf = a.buf + ((q * a.P) + p) * (int64_t)kCap;
    const int cnt = s_cnt[lq];
    if (cnt > a.kappa) {
      const uint64_t kth = block_kth(qbuf, cnt, a.kappa, sel);
      if (tid == 0) s_kept = 0;
      __syncthreads();
      for (int i = tid; i < cnt; i += 256) {
        uint64_t k = qbuf[i];
        if (k >= kth) s_stage[atomicAdd(&s_kept, 1u)] = k;
      }
      __syncthreads();
      for (int i = tid; i < a.kappa; i += 256) qbuf[i] = s_stage[i];
      __syncthreads();
    }
    if (tid == 0) a.cnt_out[q * a.P + p] = cnt < a.kappa ? cnt : a.kappa;
  }
}

// ---------------------------------------------------------------------------- merge
// Merge groups of G lists per query into one list of the kappa best keys.
// Final level: either (ids, scores) sorted by key (score desc, id asc), or, for
// a sampling scan of the cascade, only tau = the kappa-th best score (-inf when
// fewer than kappa candidates exist).
constexpr int kMergeG = 16;

__global__ __launch_bounds__(256) void k_merge(const uint64_t* __restrict__ in, const int32_t* __restrict__ in_cnt,
                                               int64_t in_stride, int L, int kappa, uint64_t* __restrict__ out,
                                               int32_t* __restrict__ out_cnt, int Lo, int32_t* __restrict__ ids,
                                               float* __restrict__ scores, float* __restrict__ tau_out) {
  __shared__ uint64_t keys[kMergeG * 256];
  __shared__ int32_t s_base[kMergeG + 1];
  __shared__ uint64_t s_stage[256];
  __shared__ uint32_t s_kept;
  __shared__ SelectSmem sel;
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x / Lo;
  const int g = blockIdx.x % Lo;
  const int l0 = g * kMergeG, l1 = min(L, l0 + kMergeG);
  if (tid == 0) {
    s_base[0] = 0;
    for (int l = l0; l < l1; ++l) s_base[l - l0 + 1] = s_base[l - l0] + in_cnt[q * L + l];
  }
  __syncthreads();
  const int total = s_base[l1 - l0];
  for (int l = l0; l < l1; ++l) {
    const uint64_t* src = in + (q * L + l) * in_stride;
    const int b = s_base[l - l0], nl = s_base[l - l0 + 1] - b;
    for (int i = tid; i < nl; i += 256) keys[b + i] = src[i];
  }
  __syncthreads();
  if (tau_out) {  // sampling scan: only the kappa-th best score matters
    float tau = -INFINITY;
    if (total >= kappa) tau = key_score(block_kth(keys, total, kappa, sel));
    if (tid == 0) tau_out[q] = tau;
    return;
  }
  int kept = total;
  if (total > kappa) {
    const uint64_t kth = block_kth(keys, total, kappa, sel);
    if (tid == 0) s_kept = 0;
    __syncthreads();
    for (int i = tid; i < total; i += 256)
      if (keys[i] >= kth) s_stage[atomicAdd(&s_kept, 1u)] = keys[i];
    __syncthreads();
    kept = kappa;
  } else {
    for (int i = tid; i < total; i += 256) s_stage[i] = keys[i];
    __syncthreads();
  }
  if (!ids) {
    uint64_t* dst = out + (q * Lo + g) * (int64_t)kappa;
    for (int i = tid; i < kept; i += 256) dst[i] = s_stage[i];
    if (tid == 0) out_cnt[q * Lo + g] = kept;
    return;
  }
  // final level: bitonic sort of 256 keys, descending (padding keys are 0)
  for (int i = tid; i < 256; i += 256)
    if (i >= kept) s_stage[i] = 0;
  __syncthreads();
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int i = tid, j = i ^ stride;
      if (j > i) {
        const bool desc = (i & size) == 0;
        uint64_t x = s_stage[i], y = s_stage[j];
        if (desc ? (x < y) : (x > y)) {
          s_stage[i] = y;
          s_stage[j] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < kappa; i += 256) {
    const uint64_t k = s_stage[i];
    ids[q * kappa + i] = (int32_t)key_id(k);
    scores[q * kappa + i] = key_score(k);
  }
}

// choose the launch shape of S2/S3 for a scan over `rows` rows
struct Shape {
  bool shared;
  int nb;
  int P;
};

Shape choose_shape(int fmt, int64_t m, int64_t rows, int C) {
  Shape sh;
  const int qpw_override = tuned_qpw();
  const int p_override = tuned_splits();
  if (qpw_override > 0) {
    sh.nb = std::max(1, std::min(4, qpw_override / 32));
    sh.shared = m <= sh.nb * 32;
  } else if (m <= 32) {
    sh = {true, 1, 0};
  } else if (m <= 64) {
    sh = {true, 2, 0};
  } else {
    sh = {false, 4, 0};
  }
  if (fmt == GV_FP32) sh.nb = 1;
  if (sh.shared && sh.nb == 4) sh.nb = 2;
  const int qwg = sh.shared ? 32 * sh.nb : 128 * sh.nb;
  const int64_t nqb = (m + qwg - 1) / qwg;
  const int rpi = sh.shared ? 128 : 32;
  const int64_t ntiles = rows / rpi + C;
  int P;
  if (p_override > 0) {
    P = p_override;
  } else {
    // about 512 workgroups in flight, at least 8 tiles per split
    int64_t want = std::max<int64_t>(8, (512 + nqb - 1) / nqb);
    P = (int)std::min<int64_t>(want, std::max<int64_t>(1, ntiles / 8));
    P = std::min(P, 1024);
  }
  if (nqb > 1 && P >= 8) P = P / 8 * 8;
  sh.P = std::max(1, P);
  return sh;
}

template <int FMT, int KSM>
gv_status launch_score(const Shape& sh, const ScoreArgs& args, hipStream_t st, unsigned grid) {
  if constexpr (FMT == GV_FP32) {
    if (sh.shared)
      hipLaunchKernelGGL((k_score_select<FMT, KSM, 1, true>), dim3(grid), dim3(256), 0, st, args);
    else
      hipLaunchKernelGGL((k_score_select<FMT, KSM, 1, false>), dim3(grid), dim3(256), 0, st, args);
  } else {
    if (sh.shared && sh.nb == 1)
      hipLaunchKernelGGL((k_score_select<FMT, KSM, 1, true>), dim3(grid), dim3(256), 0, st, args);
    else if (sh.shared)
      hipLaunchKernelGGL((k_score_select<FMT, KSM, 2, true>), dim3(grid), dim3(256), 0, st, args);
    else
      hipLaunchKernelGGL((k_score_select<FMT, KSM, 4, false>), dim3(grid), dim3(256), 0, st, args);
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
}

template <int FMT>
gv_status dispatch_ks(int ks, const Shape& sh, const ScoreArgs& args, hipStream_t st, unsigned grid) {
  if constexpr (FMT == GV_FP32) {
    if (ks <= 32) return launch_score<FMT, 32>(sh, args, st, grid);
    if (ks <= 64) return launch_score<FMT, 64>(sh, args, st, grid);
    if (ks <= 80) return launch_score<FMT, 80>(sh, args, st, grid);
    if (ks <= 128) return launch_score<FMT, 128>(sh, args, st, grid);
  } else {
    if (ks <= 4) return launch_score<FMT, 4>(sh, args, st, grid);
    if (ks <= 8) return launch_score<FMT, 8>(sh, args, st, grid);
    if (ks <= 10) return launch_score<FMT, 10>(sh, args, st, grid);
    if (ks <= 16) return launch_score<FMT, 16>(sh, args, st, grid);
  }
  set_error("reduced dimension above 256 is not supported by the scoring kernel");
  return GV_EUNSUPPORTED;
}

// sampling strides of the threshold cascade, coarsest first, ending with 1
std::vector<int> cascade(int64_t m, int64_t n, int kappa) {
  std::vector<int> s{1};
  if (m < 8) return s;
  const int64_t min_rows = 64LL * kappa;
  for (int64_t stride = 16; n / stride >= min_rows && stride <= 4096; stride *= 16) s.insert(s.begin(), (int)stride);
  return s;
}

}  // namespace

gv_status score_topk_impl(const gv_index* idx, const void* qhat, const float* t, int64_t m, int kappa,
                          int32_t* cand_ids, float* cand_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  const int fmt = idx->fmt;
  const int km = (fmt == GV_FP32) ? 2 : 16;
  const std::vector<int> levels = cascade(m, idx->n, kappa);

  // one scratch allocation sized for the largest level
  int Pmax = 1;
  for (int s : levels) Pmax = std::max(Pmax, choose_shape(fmt, m, idx->n / s, idx->C).P);
  const int64_t nl_max = m * Pmax;
  uint64_t* buf = nullptr;
  int32_t* cnt = nullptr;
  float* tau[2] = {nullptr, nullptr};
  uint64_t* lv_keys[2] = {nullptr, nullptr};
  int32_t* lv_cnt[2] = {nullptr, nullptr};
  GV_HIP(hipMallocAsync((void**)&buf, sizeof(uint64_t) * nl_max * kCap, st));
  GV_HIP(hipMallocAsync((void**)&cnt, sizeof(int32_t) * nl_max, st));
  gv_status s = GV_OK;
  if (levels.size() > 1) {
    if (hipMallocAsync((void**)&tau[0], sizeof(float) * m, st) != hipSuccess ||
        hipMallocAsync((void**)&tau[1], sizeof(float) * m, st) != hipSuccess)
      s = GV_ENOMEM;
  }
  const int Lo_max = (Pmax + kMergeG - 1) / kMergeG;
  if (s == GV_OK && Lo_max > 1) {
    for (int i = 0; i < 2; ++i)
      if (hipMallocAsync((void**)&lv_keys[i], sizeof(uint64_t) * m * Lo_max * kappa, st) != hipSuccess ||
          hipMallocAsync((void**)&lv_cnt[i], sizeof(int32_t) * m * Lo_max, st) != hipSuccess)
        s = GV_ENOMEM;
  }

  const float* tau_in = nullptr;
  for (size_t li = 0; li < levels.size() && s == GV_OK; ++li) {
    const int stride = levels[li];
    const bool last = li + 1 == levels.size();
    const Shape sh = choose_shape(fmt, m, idx->n / stride, idx->C);
    const int qwg = sh.shared ? 32 * sh.nb : 128 * sh.nb;
    const int64_t nqb = (m + qwg - 1) / qwg;
    const int P = sh.P;
    ScoreArgs args;
    args.xlow = (const uint8_t*)idx->xlow;
    args.ids = idx->ids;
    args.scale = idx->scale;
    args.offsets = idx->offsets;
    args.qhat = (const uint8_t*)qhat;
    args.qscale = t;
    args.tau_init = tau_in;
    args.buf = buf;
    args.cnt_out = cnt;
    args.m = m;
    args.C = idx->C;
    args.dp = idx->dp;
    args.ks = idx->dp / km;
    args.kappa = kappa;
    args.P = P;
    args.nqb = (int)nqb;
    args.stride = stride;
    args.xcd_map = (nqb > 1 && P % 8 == 0) ? 1 : 0;
    const int64_t grid64 = nqb * P;
    if (grid64 > 0x7fffffff) {
      s = GV_EUNSUPPORTED;
      break;
    }
    const unsigned grid = (unsigned)grid64;
    if (last) profile_mark(st, 0, true);
    switch (fmt) {
      case GV_FP32: s = dispatch_ks<GV_FP32>(args.ks, sh, args, st, grid); break;
      case GV_FP16: s = dispatch_ks<GV_FP16>(args.ks, sh, args, st, grid); break;
      case GV_BF16: s = dispatch_ks<GV_BF16>(args.ks, sh, args, st, grid); break;
      default: s = dispatch_ks<GV_FP8_E4M3>(args.ks, sh, args, st, grid); break;
    }
    if (last) profile_mark(st, 0, false);
    if (s != GV_OK) break;

    // tree merge of the m x P partial lists
    float* tau_out = last ? nullptr : tau[li & 1];
    const uint64_t* in = buf;
    const int32_t* in_cnt = cnt;
    int64_t in_stride = kCap;
    int L = P;
    int which = 0;
    if (last) profile_mark(st, 1, true);
    while (true) {
      const int Lo = (L + kMergeG - 1) / kMergeG;
      if (Lo == 1) {
        hipLaunchKernelGGL(k_merge, dim3((unsigned)m), dim3(256), 0, st, in, in_cnt, in_stride, L, kappa,
                           (uint64_t*)nullptr, (int32_t*)nullptr, 1, last ? cand_ids : (int32_t*)nullptr,
                           last ? cand_scores : (float*)nullptr, tau_out);
        break;
      }
      hipLaunchKernelGGL(k_merge, dim3((unsigned)(m * Lo)), dim3(256), 0, st, in, in_cnt, in_stride, L, kappa,
                         lv_keys[which], lv_cnt[which], Lo, (int32_t*)nullptr, (float*)nullptr, (float*)nullptr);
      in = lv_keys[which];
      in_cnt = lv_cnt[which];
      in_stride = kappa;
      L = Lo;
      which ^= 1;
    }
    if (last) profile_mark(st, 1, false);
    tau_in = tau_out;
  }
  for (int i = 0; i < 2; ++i) {
    if (lv_keys[i]) (void)hipFreeAsync(lv_keys[i], st);
    if (lv_cnt[i]) (void)hipFreeAsync(lv_cnt[i], st);
    if (tau[i]) (void)hipFreeAsync(tau[i], st);
  }
  GV_HIP(hipFreeAsync(buf, st));
  GV_HIP(hipFreeAsync(cnt, st));
  GV_TRY(s);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

// ============================================================================ S4
namespace {

__global__ __launch_bounds__(256) void k_rerank(const float* __restrict__ X, int64_t n, int D, const float* __restrict__ Q,
                                                const int32_t* __restrict__ cand, int kappa, int k,
                                                int32_t* __restrict__ out_ids, float* __restrict__ out_scores) {
  __shared__ double s_score[256];
  __shared__ int32_t s_id[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = blockIdx.x;
  const float* qv = Q + q * D;
  for (int i = tid; i < 256; i += 256) {
    s_score[i] = -INFINITY;
    s_id[i] = 0x7fffffff;
  }
  __syncthreads();
  // exact <q, x> with FP64 accumulation of exact FP32 x FP32 products
  for (int ci = wave; ci < kappa; ci += 4) {
    const int32_t id = cand[q * kappa + ci];
    if (id < 0 || id >= n) continue;  // missing candidate (e.g. non-finite query scores)
    const float* x = X + (int64_t)id * D;
    double s = 0.0;
    for (int j = lane; j < D; j += 64) s += (double)x[j] * (double)qv[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
      s_score[ci] = s;
      s_id[ci] = id;
    }
  }
  __syncthreads();
  // bitonic sort of 256 (score, id) pairs: score desc, then id asc
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
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
      __syncthreads();
    }
  }
  for (int i = tid; i < k; i += 256) {
    out_ids[q * k + i] = s_id[i];
    if (out_scores) out_scores[q * k + i] = (float)s_score[i];
  }
}

}  // namespace

gv_status rerank_impl(const gv_index* idx, const float* Q, int64_t m, const int32_t* cand, int kappa, int k,
                      int32_t* out_ids, float* out_scores, hipStream_t st) {
  if (m == 0) return GV_OK;
  hipLaunchKernelGGL(k_rerank, dim3((unsigned)m), dim3(256), 0, st, idx->X, idx->n, idx->D, Q, cand, kappa, k, out_ids,
                     out_scores);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace gv
