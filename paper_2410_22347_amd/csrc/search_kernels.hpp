// Scoring kernel of the search path (S2 + S3) and its launch helpers, shared by
// the per-format translation units that instantiate it.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "search_common.hpp"

namespace gv {
// ============================================================================ S2 + S3
//
// Work item = one wavefront = (block of 32*NB queries, one contiguous range of
// 32-row tiles).  A tile never straddles two clusters, so it meets one eager
// view q_c per query, held in registers as the matrix-core B operand.  Rows
// arrive as operand tiles (see tiled_offset): one k-step of a tile is one
// contiguous block per wavefront, and a ring of three register buffers keeps
// the next two tiles in flight while the current one is scored.  Scores leave
// the accumulators only through a threshold filter: a score below the query's
// current threshold tau can never enter the top kappa, so only survivors are
// written, as 64-bit keys (score desc, id asc), to the (query, range) buffer.
// A buffer close to full is compacted by its wavefront to the kappa best keys
// and tau rises to the kappa-th score.  Wavefronts never wait on each other.
//
// A workgroup holds four work items: four query blocks on the same rows when
// queries are many (the rows are fetched once into L1 for all four), or one
// query block on four row ranges when they are few.
//
// Threshold cascade (modes): the scan of the whole database (kMain) starts from
// a per-query seed tau that is a valid lower bound of its kappa-th best score,
// so only about kappa * 16 scores per query survive.  The seed comes from
// scans of uniform samples of the tiles (every s-th tile):
//   kDense  the sparsest sample, every score written out; a selection kernel
//           takes the kappa-th best per query;
//   kPilot  denser samples seeded by the previous level; each of R ranges keeps
//           its ceil(kappa/R) best and publishes how many it kept and the worst
//           of them: if the ranges kept kappa in total, the minimum of their
//           worst is a valid seed for the next level.
namespace scan {

constexpr int kCap = 2048;  // candidate slots per (query, range)
constexpr int kRows = kTileRows;
enum Mode { kMain = 0, kPilot = 1, kDense = 2 };

struct ScoreArgs {
  const uint8_t* xlow;    // operand tiles, n_pad x dp elements
  const int32_t* ids;     // stored row -> original id (-1: padding)
  const float* scale;     // C
  const int64_t* offsets; // C + 1 padded segment starts
  const uint8_t* qhat;    // m x C x dp, storage format
  const float* qscale;    // m x C
  const float* seed;      // m seed thresholds, or null (-inf)
  uint64_t* buf;          // m x R x kCap keys               (kMain, kPilot)
  int32_t* cnt_out;       // m x R kept per (query, range)   (kMain)
  uint32_t* tau_ord;      // m: min over ranges, ordered     (kPilot)
  int32_t* kcount;        // m: kept over ranges             (kPilot)
  float* dense;           // m x (sampled tiles * 32)        (kDense)
  int64_t m, n_pad;
  int C, dp, kappa, R, nqb, cap;
  int stride;             // scan every stride-th tile
  int xcd_map;            // 1: workgroups sharing rows are pinned to one XCD
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// kappa-th largest of the distinct keys load(0..cnt) (1 <= kappa <= cnt) by an
// MSB-first radix select with 8-bit digits, for one wavefront; returns T with
// exactly kappa keys >= T.  hist: 256 words of this wavefront's LDS.
template <typename Load>
__device__ uint64_t wave_kth(Load load, int cnt, int kappa, uint32_t* hist) {
  const int lane = threadIdx.x & 63;
  uint64_t prefix = 0, mask = 0;
  uint32_t need = (uint32_t)kappa;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = lane; b < 256; b += 64) hist[b] = 0;
    wave_sync();
    for (int i = lane; i < cnt; i += 64) {
      const uint64_t k = load(i);
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1u);
    }
    wave_sync();
    const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const uint32_t local = h0 + h1 + h2 + h3;
    uint32_t incl = local;  // keys in this lane's bins and all higher bins
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_down(incl, o);
      if (lane + o < 64) incl += v;
    }
    uint32_t a = incl - local;
    const uint32_t hb[4] = {h0, h1, h2, h3};
    int digit = -1;
    uint32_t nneed = 0, inbin = 0;
    for (int j = 3; j >= 0; --j) {
      if (a < need && need <= a + hb[j]) {
        digit = 4 * lane + j;
        nneed = need - a;
        inbin = hb[j];
      }
      a += hb[j];
    }
    const uint64_t owner = __ballot(digit >= 0);
    const int src = __ffsll((unsigned long long)owner) - 1;
    digit = __shfl(digit, src);
    nneed = __shfl(nneed, src);
    inbin = __shfl(inbin, src);
    wave_sync();
    prefix |= (uint64_t)digit << shift;
    mask |= (uint64_t)255 << shift;
    need = nneed;
    if (inbin == need) break;  // every key of this bin is in
  }
  return prefix;
}

// LDS of one wavefront
template <int QW>
struct WaveSmem {
  int32_t cnt[QW];
  float tau[QW];
  uint32_t hist[256];
  uint64_t stage[256];
  uint32_t kept;
};

// Reduce a (query, range) buffer of cnt > keep keys to its `keep` best; returns
// the smallest kept key.
template <int QW>
__device__ uint64_t wave_compact(uint64_t* qbuf, int cnt, int keep, WaveSmem<QW>& w) {
  const int lane = threadIdx.x & 63;
  // survivors were stored by other lanes of this wavefront: make them visible
  // and read them coherently from L2
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  auto load = [&](int i) { return __hip_atomic_load(qbuf + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
  const uint64_t kth = wave_kth(load, cnt, keep, w.hist);
  if (lane == 0) w.kept = 0;
  wave_sync();
  for (int i = lane; i < cnt; i += 64) {
    const uint64_t k = load(i);
    if (k >= kth) w.stage[atomicAdd(&w.kept, 1u)] = k;
  }
  wave_sync();
  for (int i = lane; i < keep; i += 64) qbuf[i] = w.stage[i];
  wave_sync();
  return kth;
}

template <int QW>
__device__ uint64_t wave_min_key(uint64_t* qbuf, int cnt, WaveSmem<QW>& w) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  auto load = [&](int i) { return __hip_atomic_load(qbuf + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
  return wave_kth(load, cnt, cnt, w.hist);
}

template <int FMT, int KS, int NB, bool SHARED, int MODE>
__global__ __launch_bounds__(256, 1) void k_score_select(ScoreArgs a) {
  using Op = MfmaOp<FMT>;
  using S = typename Op::S;
  using T = typename Op::T;
  constexpr int QW = 32 * NB;  // queries per wavefront

  __shared__ WaveSmem<QW> s_wave[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int C = a.C;
  WaveSmem<QW>& w = s_wave[wave];

  // ---- workgroup -> four (query block, range) work items
  int qb, r;
  {
    const int b = blockIdx.x;
    if (SHARED) {
      const int rgroups = a.R / 4;
      qb = b / rgroups;
      r = (b % rgroups) * 4 + wave;
    } else {
      const int qgroups = (a.nqb + 3) / 4;
      int qg, rr;
      if (a.xcd_map) {
        const int x = b & 7, j = b >> 3;
        qg = j % qgroups;
        rr = (j / qgroups) * 8 + x;
      } else {
        qg = b % qgroups;
        rr = b / qgroups;
      }
      qb = qg * 4 + wave;
      r = rr;
    }
  }
  if (qb >= a.nqb) return;  // padding work item of the last query group
  const int64_t q0 = (int64_t)qb * QW;

  for (int i = lane; i < QW; i += 64) {
    const int64_t q = q0 + i;
    w.cnt[i] = 0;
    w.tau[i] = (q < a.m) ? (a.seed ? a.seed[q] : -INFINITY) : INFINITY;
  }
  wave_sync();

  const int64_t ntiles = a.n_pad / kRows;
  const int64_t nvirt = (ntiles + a.stride - 1) / a.stride;
  const int64_t v_begin = nvirt * r / a.R, v_end = nvirt * (r + 1) / a.R;
  const int limit = a.cap - kRows;
  const int half = lane >> 5, col = lane & 31;

  if (v_begin < v_end) {
    const int64_t tile_bytes = (int64_t)kRows * a.dp * Op::EB;
    const int64_t kblock = 64 * Op::EPL * Op::EB;
    const uint8_t* xl = a.xlow + (int64_t)lane * Op::EPL * Op::EB;
    auto load_tile = [&](S (&dst)[KS], int64_t v) {
      const uint8_t* p = xl + (v < v_end ? v : v_end - 1) * a.stride * tile_bytes;
#pragma unroll
      for (int s = 0; s < KS; ++s) dst[s] = *(const S*)(p + s * kblock);
    };

    T bq[NB][KS];
    float st[NB];      // s_c * t_{q,c} for this lane's queries (times the operand widening)
    float inv_st[NB];  // 1 / st (exact: a power of two)
    float tau_s[NB];   // thresholds in the accumulator domain
    auto refresh_tau = [&]() {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) tau_s[nb] = w.tau[nb * 32 + col] * inv_st[nb];
    };

    // cluster walk: the tiles of a range are visited in increasing order
    int c;
    int64_t c_end;  // first stored row after cluster c
    {
      const int64_t row = v_begin * a.stride * kRows;
      int lo = 0, hi = C - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.offsets[mid] <= row) lo = mid; else hi = mid - 1;
      }
      c = lo;
      c_end = a.offsets[c + 1];
    }
    int cur_c = -1;
    const int64_t ns = nvirt * kRows;  // dense row count of the sample

    auto step = [&](S (&cur)[KS], S (&pf)[KS], int64_t vv) {
      load_tile(pf, vv + 2);
      const bool live = vv < v_end;
      const int64_t t = (live ? vv : v_end - 1) * a.stride;  // tile index
      const int64_t base = t * kRows;                          // its first stored row
      if (live) {
        while (base >= c_end) {
          ++c;
          c_end = a.offsets[c + 1];
        }
        if (c != cur_c) {
          cur_c = c;
          const float sc = a.scale[c] * (1.0f / (Op::kScale * Op::kScale));
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int64_t q = q0 + nb * 32 + col;
            const bool qv = q < a.m;
            const uint8_t* qp = a.qhat + ((qv ? q : 0) * C + c) * (int64_t)a.dp * Op::EB +
                                (int64_t)(half * Op::EPL) * Op::EB;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const S raw = *(const S*)(qp + (int64_t)(s * Op::KM) * Op::EB);
              bq[nb][s] = qv ? Op::cvt(raw) : zero_op<T>();
            }
            st[nb] = sc * (qv ? a.qscale[q * C + c] : 1.0f);
            inv_st[nb] = 1.0f / st[nb];
          }
          refresh_tau();
        }
      }
      f32x16 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x16{0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const T av = Op::cvt(cur[s]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = Op::mma(av, bq[nb][s], acc[nb]);
      }
      if (!live) return;
      // epilogue: lane holds query col of each block nb, tile rows (i%4) + 8*(i/4) + 4*half
      if constexpr (MODE == kDense) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int64_t q = q0 + nb * 32 + col;
          if (q >= a.m) continue;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int rt = (i & 3) + 8 * (i >> 2) + 4 * half;
            const bool real = a.ids[base + rt] >= 0;
            a.dense[q * ns + vv * kRows + rt] = real ? acc[nb][i] * st[nb] : -INFINITY;
          }
        }
        return;
      }
      bool any = false;
      float mx[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        mx[nb] = acc[nb][0];
#pragma unroll
        for (int i = 1; i < 16; ++i) mx[nb] = fmaxf(mx[nb], acc[nb][i]);
        any |= mx[nb] >= tau_s[nb];
      }
      if (__ballot(any)) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if (mx[nb] >= tau_s[nb]) {
            const int lq = nb * 32 + col;
            const int64_t q = q0 + lq;
            uint64_t* qbuf = a.buf + ((q * a.R) + r) * (int64_t)kCap;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              if (acc[nb][i] >= tau_s[nb]) {
                const int32_t id = a.ids[base + (i & 3) + 8 * (i >> 2) + 4 * half];
                if (id >= 0) {
                  const float score = acc[nb][i] * st[nb];
                  const int slot = atomicAdd(&w.cnt[lq], 1);
                  qbuf[slot] = make_key(score, (uint32_t)id);
                }
              }
            }
          }
        }
        wave_sync();
        // compaction of this wavefront's nearly full buffers
        bool full = false;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) full |= w.cnt[nb * 32 + col] > limit;
        if (__ballot(full)) {
          for (int lq = 0; lq < QW; ++lq) {
            const int cnt = w.cnt[lq];
            if (cnt <= limit) continue;
            uint64_t* qbuf = a.buf + (((q0 + lq) * a.R) + r) * (int64_t)kCap;
            const float tk = key_score(wave_compact(qbuf, cnt, a.kappa, w));
            if (lane == 0) {
              w.cnt[lq] = a.kappa;
              w.tau[lq] = fmaxf(w.tau[lq], tk);
            }
            wave_sync();
          }
          refresh_tau();
        }
      }
    };

    S b0[KS], b1[KS], b2[KS];
    load_tile(b0, v_begin);
    load_tile(b1, v_begin + 1);
    for (int64_t v = v_begin; v < v_end; v += 3) {
      step(b0, b2, v);
      step(b1, b0, v + 1);
      step(b2, b1, v + 2);
    }
  }
  if constexpr (MODE == kDense) return;

  // ---- final
  wave_sync();
  for (int lq = 0; lq < QW; ++lq) {
    const int64_t q = q0 + lq;
    if (q >= a.m) break;
    uint64_t* qbuf = a.buf + ((q * a.R) + r) * (int64_t)kCap;
    const int cnt = w.cnt[lq];
    if constexpr (MODE == kMain) {
      // keep at most kappa keys per (query, range)
      if (cnt > a.kappa) (void)wave_compact(qbuf, cnt, a.kappa, w);
      if (lane == 0) a.cnt_out[q * a.R + r] = cnt < a.kappa ? cnt : a.kappa;
    } else {
      // publish how many this range kept (at most kappa_r) and the worst of them
      if (cnt > 0) {
        const int keep = cnt < a.kappa ? cnt : a.kappa;
        const uint64_t worst = cnt > a.kappa ? wave_compact(qbuf, cnt, keep, w) : wave_min_key(qbuf, cnt, w);
        if (lane == 0) {
          atomicMin(&a.tau_ord[q], order_f32(key_score(worst)));
          atomicAdd(&a.kcount[q], keep);
        }
      }
    }
  }
}

// choose the launch shape of S2/S3 for a scan over `rows` rows
struct Shape {
  bool shared;  // the four wavefronts of a workgroup share one query block
  int nb;       // 32-query blocks per wavefront
  int R;        // row ranges per query block
  int64_t nqb;  // query blocks
  int grid;     // workgroups
  int xcd_map;
};

template <int FMT, int KS, int MODE>
void launch_score(const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  if constexpr (FMT == GV_FP32) {
    if (sh.shared)
      hipLaunchKernelGGL((k_score_select<FMT, KS, 1, true, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
    else
      hipLaunchKernelGGL((k_score_select<FMT, KS, 1, false, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
  } else {
    if (sh.shared && sh.nb == 1)
      hipLaunchKernelGGL((k_score_select<FMT, KS, 1, true, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
    else if (sh.shared)
      hipLaunchKernelGGL((k_score_select<FMT, KS, 2, true, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
    else if constexpr (KS <= 10) {
      if (sh.nb == 4)
        hipLaunchKernelGGL((k_score_select<FMT, KS, 4, false, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
      else
        hipLaunchKernelGGL((k_score_select<FMT, KS, 2, false, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
    } else {
      hipLaunchKernelGGL((k_score_select<FMT, KS, 2, false, MODE>), dim3(sh.grid), dim3(256), 0, st, args);
    }
  }
}

template <int FMT, int MODE>
gv_status dispatch_ks(int dp, const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  constexpr int km = MfmaOp<FMT>::KM;
  switch (dp / km) {
    case 32 / km: launch_score<FMT, 32 / km, MODE>(sh, args, st); break;
    case 64 / km: launch_score<FMT, 64 / km, MODE>(sh, args, st); break;
    case 128 / km: launch_score<FMT, 128 / km, MODE>(sh, args, st); break;
    case 160 / km: launch_score<FMT, 160 / km, MODE>(sh, args, st); break;
    case 192 / km: launch_score<FMT, 192 / km, MODE>(sh, args, st); break;
    case 256 / km: launch_score<FMT, 256 / km, MODE>(sh, args, st); break;
    default:
      set_error("reduced dimension above 256 is not supported by the scoring kernel");
      return GV_EUNSUPPORTED;
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace scan

// per-format entry points (search_fp32.hip, search_fp16.hip, ...)
template <int FMT, int MODE>
gv_status dispatch_scan(int dp, const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st);

}  // namespace gv
