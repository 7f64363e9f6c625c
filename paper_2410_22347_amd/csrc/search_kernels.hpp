// Scoring kernel of the search path (S2 + S3) and its launch helpers, shared by
// the per-format translation units that instantiate it.
#pragma once

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "lds_tile.hpp"
#include "search_common.hpp"

namespace gv {
// ============================================================================ S2 + S3
//
// Work item = one wavefront = (block of 32*NB queries, one contiguous range of
// 32-row tiles).  A range is walked segment by segment, a segment being the
// part of the range inside one cluster: the segment's eager views q_c are the
// matrix-core B operand and stay in registers, the tiles stream through a ring
// of P register buffers (P-1 tiles in flight while one is scored).  The
// accumulators are double-buffered so the filter of tile t-1 runs while the
// matrix core works on tile t.
//
// Filter: a score below the query's threshold tau cannot enter the top kappa,
// so only survivors leave the accumulators, as 64-bit keys (score desc, stored
// row asc) appended to the (query, range) list.  The two lanes that hold the
// same query (rows 0-3 and 4-7 of each group of eight) agree on their slots
// through one cross-half exchange; no atomics.  A list close to full is
// compacted by its wavefront to its kappa best (ordered by score desc, original
// id asc) and tau rises to the kappa-th score.  Wavefronts never wait on each
// other.
//
// A workgroup holds four work items: four query blocks on the same rows when
// queries are many (the rows are fetched once into L1/L2 for all four), or one
// query block on four row ranges when they are few.
//
// Modes: kFilter as above; kDense writes every score of a (sampled) scan to a
// dense m x ns matrix (used on the sparsest sample of the threshold cascade).
// The scan visits every stride-th tile (stride 1: the whole database).
namespace scan {

constexpr int kCap = 2048;  // key slots per (query, range) list
constexpr int kRows = kTileRows;
enum Mode { kFilter = 0, kDense = 1 };

struct ScoreArgs {
  const uint8_t* xlow;     // operand tiles, n_pad x dps elements; the scan reads the leading dp of each row
  const int32_t* ids;      // stored row -> original id (-1: padding)
  const float* scale;      // C
  const int64_t* offsets;  // C + 1 padded segment starts (stored rows)
  const int64_t* seg_end;  // C: first padding row of each segment
  const uint8_t* qhat;     // m x C x dp, view format (view_fmt of the storage format)
  const float* qscale;     // m x C
  const float* seed;       // m initial thresholds, or null (-inf)
  uint64_t* buf;           // kFilter: m x R lists of cap keys
  int32_t* cnt_out;        // kFilter: m x R list lengths
  float* dense;            // kDense: m x ns scores (ns = sampled tiles * 32)
  int64_t m, n_pad;
  int C, dp, kappa, R, nqb, cap;
  int dps;      // stored (padded) row length: tiles are 32 * dps elements apart
  int stride;   // scan every stride-th tile
  int xcd_map;  // 1: workgroups sharing rows are pinned to one XCD
  // lazy inner product (Algorithm 3): the scan projects each visited cluster's
  // view itself instead of reading qhat/qscale
  const double* lazy_A;  // C x lazy_d x lazy_D, FP64 (the model's stacked A_c)
  const float* lazy_Q;   // m x lazy_D FP32 queries
  int lazy_d, lazy_D;    // the model's reduced and full dimension
  int lazy_ds;           // leading coordinates in the view (d_search)
  // 1: a repair pass after an optimistic full scan -- only queries with a finite
  // seed are rescanned (their lists were emptied); the others' lists and
  // lengths are left as they are, and a workgroup without such a query leaves
  int repair;
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// kappa-th largest of the distinct keys load(0..cnt) (1 <= kappa <= cnt) by an
// MSB-first radix select with 8-bit digits, for one wavefront; returns T with
// exactly kappa keys >= T.  hist: 256 words of this wavefront's LDS.  UNROLL
// keys per lane are loaded before any is counted (loads from global memory
// then overlap instead of each waiting for the last).
template <int UNROLL = 1, typename Load>
__device__ uint64_t wave_kth(Load load, int cnt, int kappa, uint32_t* hist) {
  const int lane = threadIdx.x & 63;
  uint64_t prefix = 0, mask = 0;
  uint32_t need = (uint32_t)kappa;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = lane; b < 256; b += 64) hist[b] = 0;
    wave_sync();
    for (int i0 = lane; i0 < cnt; i0 += 64 * UNROLL) {
      uint64_t k[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) k[u] = i0 + 64 * u < cnt ? load(i0 + 64 * u) : 0;
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        if (i0 + 64 * u < cnt && (k[u] & mask) == prefix) atomicAdd(&hist[(k[u] >> shift) & 255], 1u);
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

// LDS of one wavefront; CAPL = largest list a compaction stages
template <int QW, int CAPL>
struct WaveSmem {
  float tau[QW];
  uint32_t hist[256];
  uint32_t kept;
  uint64_t idk[CAPL];  // compaction: the list's keys
};

// ---- LDS of one workgroup: four wavefronts' staging (WaveSmem) and the tile
// ring.  A CU has 160 KiB, so two workgroups per CU take at most 80 KiB each.
constexpr int wave_smem_bytes(int qw, int capl) { return (qw * 4 + 256 * 4 + 4 + 7) / 8 * 8 + 8 * capl; }
constexpr int lds_budget(int occ) { return 160 * 1024 / occ - 256; }  // some room for the queue kernel's own words
template <int FMT, int KS>
constexpr int ring_tile_bytes() { return KS * 64 * MfmaOp<FMT>::EPL * MfmaOp<FMT>::EB; }
// tiles of a ring shared by two workgroups per CU: the deepest ring, up to five
// tiles (the copies of three tiles in flight while one is scored), that fits
// beside a 768-key staging; three is the fewest the pipeline needs
template <int FMT, int KS, int NB>
constexpr int ring_tiles_two_per_cu() {
  for (int pl = 5; pl > 3; --pl)
    if (4 * wave_smem_bytes(32 * NB, 768) + pl * ring_tile_bytes<FMT, KS>() <= lds_budget(2)) return pl;
  return 3;
}
// keys a compaction can stage: the whole list with one workgroup per CU and no
// ring; else half a list where it fits beside the ring, or 768 keys
template <int FMT, int KS, int NB, int OCC, bool WGT, int PL>
constexpr int staging_keys() {
  if (!(OCC >= 2 || WGT)) return kCap;
  const int ring = WGT ? PL * ring_tile_bytes<FMT, KS>() : 16;
  return 4 * wave_smem_bytes(32 * NB, kCap / 2) + ring <= lds_budget(OCC) ? kCap / 2 : 768;
}

// Reduce the list L of n keys (n > keep), keyed (score desc, stored row asc),
// so that it still holds the `keep` best by (score desc, original id asc).
// Usual case: every key whose score reaches the keep-th best score stays (ties
// at that score included, whatever their ids), no id is looked up, and the new
// length is returned if it is at most `room`.  Otherwise the keys are re-keyed
// by original id and exactly `keep` stay.  *tk: the keep-th best score.
template <typename W>
__device__ int compact_list(uint64_t* L, int n, int keep, int room, const int32_t* __restrict__ ids, W& w,
                            float* tk) {
  const int lane = threadIdx.x & 63;
  // the keys were stored by lanes of this wavefront: make them visible and
  // read them coherently from L2, four loads in flight per lane
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  for (int i0 = 0; i0 < n; i0 += 256) {
    uint64_t k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 64 + lane;
      k[u] = i < n ? __hip_atomic_load(L + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 64 + lane;
      if (i < n) w.idk[i] = k[u];
    }
  }
  wave_sync();
  const uint64_t kth = wave_kth([&](int i) { return w.idk[i]; }, n, keep, w.hist);
  *tk = key_score(kth);
  const uint64_t lo = kth & 0xFFFFFFFF00000000ull;  // smallest key with the keep-th best score
  int c = 0;
  for (int i = lane; i < n; i += 64) c += w.idk[i] >= lo;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (c <= room) {
    if (lane == 0) w.kept = 0;
    wave_sync();
    for (int i = lane; i < n; i += 64) {
      const uint64_t k = w.idk[i];
      if (k >= lo) L[atomicAdd(&w.kept, 1u)] = k;
    }
    wave_sync();
    return c;
  }
  // many ties at the keep-th best score: exact reduction by original id (the
  // id of each key is looked up where it is compared; this path is rare)
  auto by_id = [&](uint64_t k) {
    const uint32_t row = 0xFFFFFFFFu - (uint32_t)k;
    return (k & 0xFFFFFFFF00000000ull) | (uint64_t)(0xFFFFFFFFu - (uint32_t)ids[row]);
  };
  const uint64_t kid = wave_kth([&](int i) { return by_id(w.idk[i]); }, n, keep, w.hist);
  if (lane == 0) w.kept = 0;
  wave_sync();
  for (int i = lane; i < n; i += 64) {
    const uint64_t k = w.idk[i];
    if (by_id(k) >= kid) L[atomicAdd(&w.kept, 1u)] = k;
  }
  wave_sync();
  return keep;
}

// cluster of stored row `row`: the number of j in [1, C) with offsets[j] <= row
// (segments are contiguous and increasing; empty ones are skipped)
__device__ inline int find_cluster(const int64_t* __restrict__ offsets, int C, int64_t row) {
  const int lane = threadIdx.x & 63;
  int c = 0;
  for (int j0 = 1; j0 < C; j0 += 64) {
    const int j = j0 + lane;
    const bool le = j < C && offsets[j] <= row;
    c += __popcll(__ballot(le));
  }
  return c;
}

// a wavefront-uniform value computed in vector registers, made scalar
__device__ inline int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline float uniformf(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

// s_waitcnt vmcnt(N): at most N vector memory operations of this wavefront
// still outstanding (gfx9 encoding; expcnt and lgkmcnt not waited for)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// workgroup barrier without a memory fence: the compiler keeps memory
// operations on their side of it, the hardware adds no waits
__device__ __forceinline__ void block_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// k-step operand sets held in registers on the LDS ring: the smallest divisor
// of the tile's k-steps that is at least 4 (all of them below 4)
constexpr int window_steps(int ks) {
  for (int w = 4; w < ks; ++w)
    if (ks % w == 0) return w;
  return ks;
}

// compile-time unrolled loop: f(std::integral_constant<int, i>) for i in [I, N)
template <int I, int N>
struct Unroll {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      Unroll<I + 1, N>::run(f);
    }
  }
};

// value of x in the lane 32 apart (lanes l and l ^ 32 exchange)
__device__ inline int other_half(int x) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  return (int)((threadIdx.x & 32) ? r[0] : r[1]);
}

__device__ inline float max16(const f32x16& v) {
  float a = fmaxf(fmaxf(v[0], v[1]), v[2]);
  float b = fmaxf(fmaxf(v[3], v[4]), v[5]);
  float c = fmaxf(fmaxf(v[6], v[7]), v[8]);
  float d = fmaxf(fmaxf(v[9], v[10]), v[11]);
  float e = fmaxf(fmaxf(v[12], v[13]), v[14]);
  return fmaxf(fmaxf(fmaxf(a, b), fmaxf(c, d)), fmaxf(e, v[15]));
}

// tile row of accumulator element i for a lane of half h (v_mfma_f32_32x32x*
// output layout: rows (i % 4) + 8 * (i / 4) + 4 * h, column = lane % 32)
__device__ constexpr int acc_row(int i, int h) { return (i & 3) + 8 * (i >> 2) + 4 * h; }

// The view of one query for cluster c as the lazy inner product computes it
// (Algorithm 3, the projection A_c q made where the cluster is visited):
// v_j = fl32(A_c(j, :) q) with FP64 accumulation (lane-strided sums, butterfly
// reduction, lane 0's value -- the same arithmetic as the eager projection of
// small batches), t = the power of two putting max |v_j| (j < ds) into
// (T/2, T], and the FP16 view rnd(v_j / t) for j < ds, zero up to dp.
// One wavefront; writes dp halves to view[] and returns t.
__device__ inline float lazy_view(const double* __restrict__ A, const float* __restrict__ q, int c, int d, int D,
                                  int ds, int dp, uint16_t* view) {
  const int lane = threadIdx.x & 63;
  const double* Ac = A + (int64_t)c * d * D;
  float amax = 0.0f;
  float vals[4];  // dp <= 256: lane l keeps v_j for j = 64 u + l
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    vals[u] = 0.0f;
    for (int jj = 0; jj < 64 && 64 * u + jj < ds; ++jj) {
      const double* a = Ac + (int64_t)(64 * u + jj) * D;
      double sacc = 0.0;
      for (int k = lane; k < D; k += 64) sacc += a[k] * (double)q[k];
      for (int o = 32; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o);
      const float v = (float)__shfl(sacc, 0);  // lane 0's sum, as the eager projection keeps
      if (jj == lane) vals[u] = v;
      amax = fmaxf(amax, fabsf(v));
    }
  }
  const float t = pow2_scale(amax, 65504.0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = u * 64 + lane;
    if (j < dp) view[j] = j < ds ? to_fp16((double)vals[u] / (double)t) : (uint16_t)0;
  }
  return t;
}

// The scan of one workgroup-sized piece b of a launch (four work items), shared
// by the one-search kernel (b = blockIdx.x) and the persistent kernel that
// pulls pieces of several searches from a queue.
template <int FMT, int KS, int NB, bool SHARED, int MODE, int P, bool DEFER, int OCC, bool FULL, bool WGT, int PL,
          bool LAZY>
__device__ __forceinline__ void scan_body(const ScoreArgs& a, const int b_item) {
  using Op = MfmaOp<FMT>;
  using S = typename Op::S;
  using T = typename Op::T;
  constexpr int QW = 32 * NB;  // queries per wavefront
  // unrolled steps per loop iteration (ring x accumulator parity); the
  // workgroup-shared ring (WGT) advances one tile per step with the filter deferred
  constexpr int U = WGT ? 2 : (DEFER ? 2 * P : P);
  constexpr int kblock_c = 64 * Op::EPL * Op::EB;  // bytes of one k-step block of a tile
  constexpr int TB = KS * kblock_c;                 // bytes of one tile

  // two workgroups per CU, or an LDS tile ring, need the smaller compaction staging
  // (KernelCfg states the same constants for the host-side plan checks)
  constexpr int CAPL = staging_keys<FMT, KS, NB, OCC, WGT, PL>();
  static_assert(CAPL - kRows * (U + 1) >= 256 + kRows, "the staging must hold kappa <= 256 plus a tile");
  static_assert(sizeof(WaveSmem<QW, CAPL>) == wave_smem_bytes(QW, CAPL), "staging size as planned");
  static_assert(TB == ring_tile_bytes<FMT, KS>(), "tile size as planned");
  static_assert(4 * sizeof(WaveSmem<QW, CAPL>) + (WGT ? PL * TB : 16) + (LAZY ? 4 * QW * KS * 16 * 2 + 16 * QW : 32) <=
                    lds_budget(OCC),
                "the workgroup's LDS must allow OCC workgroups per CU");
  __shared__ WaveSmem<QW, CAPL> s_wave[4];
  __shared__ __attribute__((aligned(16))) uint8_t s_ring[WGT ? PL * TB : 16];
  // lazy views: per wavefront, its queries' FP16 views of the visited cluster
  static_assert(!LAZY || (FMT == GV_FP16 && SHARED && NB == 1), "lazy views: FP16 storage, one shared query block");
  __shared__ __attribute__((aligned(16))) uint16_t s_lazy[LAZY ? 4 * QW * KS * 16 : 8];
  __shared__ float s_lazy_t[LAZY ? 4 * QW : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  WaveSmem<QW, CAPL>& w = s_wave[wave];

  // ---- workgroup -> four (query block, range) work items
  int qb, r;
  {
    const int b = b_item;
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
  if (a.repair) {  // the same branch for the whole workgroup (a kernel argument)
    __shared__ int s_need;
    if (threadIdx.x == 0) s_need = 0;
    __syncthreads();
    bool need = false;
    if (qb < a.nqb)
      for (int i = lane; i < QW; i += 64) {
        const int64_t q = (int64_t)qb * QW + i;
        need |= q < a.m && a.seed[q] < INFINITY;
      }
    if (__ballot(need) != 0 && lane == 0) atomicOr(&s_need, 1);
    __syncthreads();
    if (s_need == 0) return;
  }
  // padding work item of the last query group (with a shared tile ring it still
  // loads its share of the tiles and meets every barrier; its queries are void)
  if (!WGT && qb >= a.nqb) return;
  const int64_t q0 = (int64_t)qb * QW;

  for (int i = lane; i < QW; i += 64) {
    const int64_t q = q0 + i;
    w.tau[i] = (q < a.m) ? (a.seed ? a.seed[q] : -INFINITY) : INFINITY;
  }
  wave_sync();

  const int64_t stride = FULL ? 1 : a.stride;  // FULL: the scan of the whole database
  const int64_t ntiles = a.n_pad / kRows;
  const int64_t nvirt = (ntiles + stride - 1) / stride;
  const int64_t v_begin = nvirt * r / a.R, v_end = nvirt * (r + 1) / a.R;
  const int64_t ns = nvirt * kRows;  // dense: row count of the sample
  // a list takes at most 32 keys per tile; between two overflow checks at most
  // U + 1 tiles; a compaction stages the whole list in this wavefront's LDS,
  // which holds CAPL keys (fewer than the list capacity with an LDS tile ring)
  const int lim = (a.cap < CAPL ? a.cap : CAPL) - kRows * (U + 1);
  // a compaction that keeps ties may leave at most this many keys (else it is exact)
  const int room = (lim + a.kappa) / 2;

  int cnt[NB];
  int64_t lbase[NB];  // first key slot of this lane's (query, range) list
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    cnt[nb] = 0;
    const int64_t q = q0 + nb * 32 + col;
    lbase[nb] = ((q < a.m ? q : 0) * a.R + r) * (int64_t)a.cap;
  }

  const int64_t tile_bytes = (int64_t)kRows * a.dps * Op::EB;
  const int64_t kblock = 64 * Op::EPL * Op::EB;
  const uint8_t* xl = a.xlow + (int64_t)lane * Op::EPL * Op::EB;

  T bq[NB][KS];
  float st[NB];      // s_c * t_{q,c} for this lane's queries (times the operand widening)
  float inv_st[NB];  // 1 / st (exact: a power of two)
  float tau_s[NB];   // thresholds in the accumulator domain

  // --------------------------------------------------------------- epilogue
  // Padding rows of a segment's last tile never survive (NaN fails every compare).
  auto mask_padding = [&](f32x16 (&A)[NB], int64_t base, int64_t real_end) __attribute__((always_inline)) {
    Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
      constexpr int nb = decltype(nbc)::value;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (base + acc_row(i, half) >= real_end) A[nb][i] = __builtin_nanf("");
    });
  };

  // Threshold filter of one scored tile.  mx[nb]: the largest of this lane's 16
  // scores of query block nb, padding rows included (they are masked here, on
  // the rare path).  Survivors are appended to the lane's list as keys; the two
  // lanes holding one query agree on their slots through one lane swap.
  auto filter = [&](f32x16 (&A)[NB], int64_t vt, int64_t real_end, const float (&mx)[NB], bool valid)
      __attribute__((always_inline)) {
    bool any = false;
    Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
      constexpr int nb = decltype(nbc)::value;
      any |= mx[nb] >= tau_s[nb];
    });
    any = any && valid;  // the maxima are taken unconditionally, beside the matrix core
    if (__ballot(any) == 0) return;
    const int64_t base = vt * stride * kRows;  // first stored row of the tile
    if (base + kRows > real_end) mask_padding(A, base, real_end);
    Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
      constexpr int nb = decltype(nbc)::value;
      const float t = tau_s[nb];
      if (__ballot(mx[nb] >= t) == 0) return;
      uint32_t mask = 0;  // survivors among this lane's 16 scores
#pragma unroll
      for (int i = 0; i < 16; ++i) mask |= A[nb][i] >= t ? (1u << i) : 0u;
      const int p = __builtin_popcount(mask);
      const int pp = other_half(p);  // the other lane holding this query
      int64_t o = lbase[nb] + cnt[nb] + (half ? pp : 0);  // list slot of this lane's first survivor
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (mask & (1u << i)) {
          a.buf[o] = make_key(A[nb][i] * st[nb], (uint32_t)(base + acc_row(i, half)));
          ++o;
        }
      }
      cnt[nb] += p + pp;
    });
  };

  // every score of one tile, for the dense sample
  auto dense_out = [&](f32x16 (&A)[NB], int64_t vt, int64_t real_end) __attribute__((always_inline)) {
    const int64_t base = vt * stride * kRows;
    if (base + kRows > real_end) mask_padding(A, base, real_end);
    Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
      constexpr int nb = decltype(nbc)::value;
      const int64_t q = q0 + nb * 32 + col;
      if (q < a.m) {
        float* drow = a.dense + q * ns + vt * kRows;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float v = A[nb][i];
          drow[acc_row(i, half)] = (v == v) ? v * st[nb] : -INFINITY;
        }
      }
    });
  };

  // filter (or dense output) of a tile whose maxima are not yet known
  auto epilogue = [&](f32x16 (&A)[NB], int64_t vt, int64_t real_end) __attribute__((always_inline)) {
    if constexpr (MODE == kDense) {
      dense_out(A, vt, real_end);
    } else {
      float mx[NB];
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) { mx[decltype(nbc)::value] = max16(A[decltype(nbc)::value]); });
      filter(A, vt, real_end, mx, true);
    }
  };

  // --------------------------------------------------------------- overflow
  auto check_overflow = [&]() __attribute__((always_inline)) {
    if constexpr (MODE == kFilter) {
      bool full = false;
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) { full |= cnt[decltype(nbc)::value] > lim; });
      if (__ballot(full) == 0) return;
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
        constexpr int nb = decltype(nbc)::value;
        uint64_t fm = __ballot(cnt[nb] > lim) & 0xFFFFFFFFull;
        while (fm) {
          const int cc = __ffsll((unsigned long long)fm) - 1;
          fm &= fm - 1;
          const int n = __shfl(cnt[nb], cc);
          const int64_t lb = __shfl(lbase[nb], cc);
          float tk;
          const int kept = compact_list(a.buf + lb, n, a.kappa, room, a.ids, w, &tk);
          const int lq = nb * 32 + cc;
          if (lane == 0) w.tau[lq] = fmaxf(w.tau[lq], tk);
          wave_sync();
          if (col == cc) {
            cnt[nb] = kept;
            tau_s[nb] = w.tau[lq] * inv_st[nb];
          }
        }
      });
    }
  };

  // --------------------------------------------------------------- segments
  int64_t v = v_begin;
  while (v < v_end) {
    const int64_t row0 = v * stride * kRows;
    const int c = find_cluster(a.offsets, a.C, row0);
    const int64_t tiles_end = uniform64(a.offsets[c + 1]) / kRows;  // first tile after the segment
    const int64_t v1 = std::min<int64_t>(v_end, (tiles_end + stride - 1) / stride);
    const int64_t real_end = uniform64(a.seg_end[c]);
    if constexpr (LAZY) {
      // Algorithm 3: the views of this cluster are made here, for the block's
      // queries, into this wavefront's LDS, then taken as the eager views are
      constexpr int DP = KS * 16;
      uint16_t* vw = s_lazy + wave * QW * DP;
      const int64_t nq = std::min<int64_t>(QW, a.m - q0);
      for (int i = 0; i < nq; ++i) {
        const float t = lazy_view(a.lazy_A, a.lazy_Q + (q0 + i) * a.lazy_D, c, a.lazy_d, a.lazy_D, a.lazy_ds, DP,
                                  vw + i * DP);
        if (lane == 0) s_lazy_t[wave * QW + i] = t;
      }
      wave_sync();
      const float sc = uniformf(a.scale[c]) * (1.0f / Op::kScale);
      const int64_t q = q0 + col;
      const bool qv = q < a.m;
      const uint16_t* qp = vw + (qv ? col : 0) * DP + half * Op::EPL;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const typename Op::QS raw = *(const typename Op::QS*)(qp + s * Op::KM);
        bq[0][s] = qv ? raw : zero_op<T>();
      }
      st[0] = sc * (qv ? s_lazy_t[wave * QW + col] : 1.0f);
      inv_st[0] = 1.0f / st[0];
      tau_s[0] = w.tau[col] * inv_st[0];
      wave_sync();  // the views are in registers before the next segment rewrites them
    } else {
      const float sc = uniformf(a.scale[c]) * (1.0f / Op::kScale);
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
        constexpr int nb = decltype(nbc)::value;
        const int64_t q = q0 + nb * 32 + col;
        const bool qv = q < a.m;
        const uint8_t* qp = a.qhat + ((qv ? q : 0) * a.C + c) * (int64_t)a.dp * Op::QEB +
                            (int64_t)(half * Op::EPL) * Op::QEB;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const typename Op::QS raw = *(const typename Op::QS*)(qp + (int64_t)(s * Op::KM) * Op::QEB);
          bq[nb][s] = qv ? raw : zero_op<T>();
        }
        st[nb] = sc * (qv ? a.qscale[q * a.C + c] : 1.0f);
        inv_st[nb] = 1.0f / st[nb];
        tau_s[nb] = w.tau[nb * 32 + col] * inv_st[nb];
      });
    }

    const int64_t v0 = v;
    auto load_tile = [&](S (&dst)[KS], int64_t vv) __attribute__((always_inline)) {
      const uint8_t* p = xl + (vv < v1 ? vv : v1 - 1) * stride * tile_bytes;
#pragma unroll
      for (int s = 0; s < KS; ++s) dst[s] = *(const S*)(p + s * kblock);
    };
    // LDS tile ring: the k-step operands pass through a window of LW register
    // sets.  K-step s of tile t sits in win[s % LW]; once consumed, its set
    // takes k-step s + LW, of tile t or, past the tile's end, k-step
    // s + LW - KS of tile t + 1 -- the same set since LW divides KS.  (LW sets
    // instead of a whole tile keep two wavefronts per SIMD within 256
    // registers; LW k-steps of matrix-core work cover an LDS read.)
    constexpr int LW = WGT ? window_steps(KS) : KS;
    static_assert(KS % LW == 0, "the window must divide the tile's k-steps");
    auto refill = [&](S (&win)[LW], auto stc, const uint8_t* cur_p, const uint8_t* nxt_p) __attribute__((always_inline)) {
      constexpr int st_ = decltype(stc)::value;
      constexpr int nx = st_ + LW;
      if constexpr (nx < KS) win[st_ % LW] = *(const S*)(cur_p + nx * kblock_c);
      else win[st_ % LW] = *(const S*)(nxt_p + (nx - KS) * kblock_c);
    };
    // matrix-core chain of one tile with the maxima of the previous tile's
    // scores (Pv) computed between its steps: the vector ALU work runs while
    // the matrix core is busy instead of after it.  src: the tile's operands
    // (register ring), or the LDS ring's window with the tile's and the next
    // tile's slots (cur_p, nxt_p)
    auto mma_tile_max = [&](auto& src, f32x16 (&A)[NB], const f32x16 (&Pv)[NB], float (&mx)[NB],
                            const uint8_t* cur_p, const uint8_t* nxt_p) __attribute__((always_inline)) {
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
        constexpr int nb = decltype(nbc)::value;
        A[nb] = f32x16{0};
        mx[nb] = Pv[nb][0];
      });
      Unroll<0, KS>::run([&](auto sc) __attribute__((always_inline)) {
        constexpr int st_ = decltype(sc)::value;
        const T av = Op::cvt(src[WGT ? st_ % LW : st_]);
        Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
          constexpr int nb = decltype(nbc)::value;
          A[nb] = Op::mma(av, bq[nb][st_], A[nb]);
        });
        if constexpr (WGT) refill(src, sc, cur_p, nxt_p);
        constexpr int j0 = 1 + st_ * 15 / KS, j1 = 1 + (st_ + 1) * 15 / KS;
        Unroll<j0, j1>::run([&](auto jc) __attribute__((always_inline)) {
          constexpr int j = decltype(jc)::value;
          Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
            constexpr int nb = decltype(nbc)::value;
            mx[nb] = fmaxf(mx[nb], Pv[nb][j]);
          });
        });
      });
      Unroll<0, KS>::run([&](auto) __attribute__((always_inline)) {
        Unroll<0, NB>::run([&](auto) __attribute__((always_inline)) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix-core op
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then up to two vector ALU ops
        });
        if constexpr (WGT) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // the refill of the k-step
      });
    };
    auto mma_tile = [&](const S (&src)[KS], f32x16 (&A)[NB]) __attribute__((always_inline)) {
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) { A[decltype(nbc)::value] = f32x16{0}; });
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const T av = Op::cvt(src[s]);
        Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
          constexpr int nb = decltype(nbc)::value;
          A[nb] = Op::mma(av, bq[nb][s], A[nb]);
        });
      }
    };
    // the same through the LDS ring's window
    auto mma_tile_win = [&](S (&win)[LW], f32x16 (&A)[NB], const uint8_t* cur_p, const uint8_t* nxt_p)
        __attribute__((always_inline)) {
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) { A[decltype(nbc)::value] = f32x16{0}; });
      Unroll<0, KS>::run([&](auto sc) __attribute__((always_inline)) {
        constexpr int st_ = decltype(sc)::value;
        const T av = Op::cvt(win[st_ % LW]);
        Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
          constexpr int nb = decltype(nbc)::value;
          A[nb] = Op::mma(av, bq[nb][st_], A[nb]);
        });
        refill(win, sc, cur_p, nxt_p);
      });
    };

    if constexpr (WGT) {
      // ---- tiles shared by the workgroup through an LDS ring of PL tiles.  Each
      // wavefront copies every fourth 1 KiB chunk of a tile straight to LDS
      // (asm copies: the compiler does not order LDS reads behind them); after
      // its own copies of a tile land (memory counter) and a barrier, every
      // wavefront may read the whole tile.  Vector memory operations complete
      // in order, so "at most N outstanding", N = the copies issued after the
      // tile's, is met only once the tile's copies have landed.  Survivor
      // stores issued in between count too: the wait is then longer than
      // needed, never shorter.  Each k-step's operands are read from the ring
      // LW k-steps before their matrix-core ops, so a tile's slot is read while
      // that tile and the one before it are scored; a wavefront has received
      // every read of a tile before it reaches the barrier after that tile.
      static_assert(TB % 1024 == 0, "tiles are copied in 1 KiB chunks");
      constexpr int NCH = TB / 1024;
      constexpr int SH_HI = (NCH + 3) / 4, SH_LO = NCH / 4;
      static_assert(PL >= 3, "the ring holds the tile in use, the next one and one in flight");
      const int wv = __builtin_amdgcn_readfirstlane(wave);  // this wavefront's index, in a scalar register
      const bool hi = wv < (NCH & 3);
      const uint32_t ring_lds = (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint8_t*)s_ring);
      const uint8_t* ring_lane = s_ring + lane * Op::EPL * Op::EB;  // this lane's operands in slot 0
      int slot_in = 0;  // ring slot of the next tile to copy
      auto issue = [&](int64_t vv) __attribute__((always_inline)) {
        const int64_t vc = vv < v1 ? vv : v1 - 1;
        const uint8_t* g = a.xlow + vc * stride * tile_bytes + (int64_t)lane * 16;
        const uint32_t ls = ring_lds + (uint32_t)(slot_in * TB);
        Unroll<0, SH_HI>::run([&](auto kc) __attribute__((always_inline)) {
          const int j = wv + 4 * decltype(kc)::value;
          if (j < NCH) copy_lds16(g + j * 1024, ls + (uint32_t)(j * 1024));
        });
        slot_in = slot_in + 1 == PL ? 0 : slot_in + 1;
      };
      // own copies of a tile have landed while those of `later` newer tiles may
      // still be in flight; then the barrier makes every wavefront's copies visible
      auto arrive = [&](auto laterc) __attribute__((always_inline)) {
        constexpr int later = decltype(laterc)::value;
        if (hi) wait_vm<later * SH_HI>(); else wait_vm<later * SH_LO>();
        block_barrier();
      };
      Unroll<0, PL - 1>::run([&](auto pc) __attribute__((always_inline)) { issue(v0 + decltype(pc)::value); });
      arrive(std::integral_constant<int, PL - 2>{});
      f32x16 acc0[NB], acc1[NB];
      S win[LW];
#pragma unroll
      for (int s = 0; s < LW; ++s) win[s] = *(const S*)(ring_lane + s * kblock_c);
      int slot_rd = 1;  // ring slot of the next tile
      int slot_cur = 0;  // ring slot of the tile being scored
      for (int64_t vb = v0; vb < v1; vb += 2) {
        Unroll<0, 2>::run([&](auto uc) __attribute__((always_inline)) {
          constexpr int u = decltype(uc)::value;
          const int64_t vt = vb + u;
          if (vt >= v1) return;
          if (vt + 1 < v1) {
            // tile vt + 1 has landed once the copies of at most PL - 3 newer
            // tiles are in flight; after the barrier every wavefront is done
            // with tile vt - 1, whose slot takes the next copy
            arrive(std::integral_constant<int, PL - 3>{});
            issue(vt + PL - 1);
          }
          // the matrix-core chain of tile vt reads the rest of tile vt and the
          // first LW k-steps of tile vt + 1 (after the last tile those reads
          // are discarded)
          const uint8_t* curp = ring_lane + slot_cur * TB;
          const uint8_t* nxt = ring_lane + slot_rd * TB;
          slot_cur = slot_rd;
          slot_rd = slot_rd + 1 == PL ? 0 : slot_rd + 1;
          if constexpr (MODE == kFilter) {
            float mx[NB];
            if constexpr (u & 1) mma_tile_max(win, acc1, acc0, mx, curp, nxt); else mma_tile_max(win, acc0, acc1, mx, curp, nxt);
            if constexpr (u & 1) filter(acc0, vt - 1, real_end, mx, vt > v0); else filter(acc1, vt - 1, real_end, mx, vt > v0);
          } else {
            if constexpr (u & 1) mma_tile_win(win, acc1, curp, nxt); else mma_tile_win(win, acc0, curp, nxt);
            if (vt > v0) {
              if constexpr (u & 1) epilogue(acc0, vt - 1, real_end); else epilogue(acc1, vt - 1, real_end);
            }
          }
        });
        check_overflow();
      }
      if ((v1 - 1 - v0) & 1) epilogue(acc1, v1 - 1, real_end); else epilogue(acc0, v1 - 1, real_end);
      check_overflow();
      wait_vm<0>();  // the tail copies land before the ring is reused
      block_barrier();
    } else {
      S ring[P][KS];
      Unroll<0, P - 1>::run([&](auto pc) __attribute__((always_inline)) { load_tile(ring[decltype(pc)::value], v0 + decltype(pc)::value); });
      f32x16 acc0[NB], acc1[NB];
  
      for (int64_t vb = v0; vb < v1; vb += U) {
        // Loads and matrix-core steps run unconditionally (tiles past the
        // segment re-read its last tile and are not filtered), so the memory
        // counter waits are the same on every path through the loop.
        Unroll<0, U>::run([&](auto uc) __attribute__((always_inline)) {
          constexpr int u = decltype(uc)::value;
          const int64_t vt = vb + u;
          load_tile(ring[(u + P - 1) % P], vt + P - 1);
          if constexpr (DEFER && MODE == kFilter) {
            // matrix core on tile vt, beside it the maxima of tile vt - 1, then its filter
            float mx[NB];
            if constexpr (u & 1) mma_tile_max(ring[u % P], acc1, acc0, mx, nullptr, nullptr); else mma_tile_max(ring[u % P], acc0, acc1, mx, nullptr, nullptr);
            const bool valid = (u > 0 || vt > v0) && vt - 1 < v1;
            if constexpr (u & 1) filter(acc0, vt - 1, real_end, mx, valid); else filter(acc1, vt - 1, real_end, mx, valid);
          } else if constexpr (DEFER) {
            if constexpr (u & 1) mma_tile(ring[u % P], acc1); else mma_tile(ring[u % P], acc0);
            if ((u > 0 || vt > v0) && vt - 1 < v1) {
              if constexpr (u & 1) epilogue(acc0, vt - 1, real_end); else epilogue(acc1, vt - 1, real_end);
            }
          } else {
            mma_tile(ring[u % P], acc0);
            if (vt < v1) epilogue(acc0, vt, real_end);
          }
        });
        check_overflow();
      }
      if constexpr (DEFER) {  // the last tile's filter, when the final step scored a real tile
        if ((v1 - v0) % U == 0) {
          epilogue(acc1, v1 - 1, real_end);  // U is even: the final step used acc1
          check_overflow();
        }
      }
    }
    v = v1;
  }

  if constexpr (MODE == kFilter) {
    if (half == 0) {
      Unroll<0, NB>::run([&](auto nbc) __attribute__((always_inline)) {
        constexpr int nb = decltype(nbc)::value;
        const int64_t q = q0 + nb * 32 + col;
        if (q < a.m && (!a.repair || a.seed[q] < INFINITY)) a.cnt_out[q * a.R + r] = cnt[nb];
      });
    }
  }
}

template <int FMT, int KS, int NB, bool SHARED, int MODE, int P, bool DEFER, int OCC, bool FULL, bool WGT, int PL,
          bool LAZY = false>
__global__ __launch_bounds__(256, OCC) void k_scan(ScoreArgs a) {
  scan_body<FMT, KS, NB, SHARED, MODE, P, DEFER, OCC, FULL, WGT, PL, LAZY>(a, blockIdx.x);
}

// The repair pass of an optimistic full scan (a.repair = 1): the same scan,
// under its own name so that kernel traces keep the two launches apart.
template <int FMT, int KS, int NB, bool SHARED, int P, bool DEFER, int OCC, bool WGT, int PL, bool LAZY = false>
__global__ __launch_bounds__(256, OCC) void k_scan_repair(ScoreArgs a) {
  scan_body<FMT, KS, NB, SHARED, kFilter, P, DEFER, OCC, true, WGT, PL, LAZY>(a, blockIdx.x);
}

// Persistent form: workgroups pull pieces (c, b) -- search c, piece b of its
// launch grid -- from one queue over several searches that share this
// instantiation, until the queue is drained.  off[c] is the first queue index
// of search c (off[ncoll] = all pieces); *head starts at 0.  Every workgroup
// leaves once the head passes the end, so the grid drains.
template <int FMT, int KS, int NB, bool SHARED, int MODE, int P, bool DEFER, int OCC, bool FULL, bool WGT, int PL>
__global__ __launch_bounds__(256, OCC) void k_scan_queue(const ScoreArgs* __restrict__ args,
                                                         const int64_t* __restrict__ off, int ncoll,
                                                         int* __restrict__ head) {
  __shared__ int s_item;
  const int64_t total = off[ncoll];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    __syncthreads();
    const int64_t it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: the search's arguments load as scalars
    __syncthreads();  // every wave has the item before thread 0 takes the next one
    if (it >= total) break;
    int c = 0;
    while (c + 1 < ncoll && off[c + 1] <= it) ++c;
    const ScoreArgs a = args[c];
    scan_body<FMT, KS, NB, SHARED, MODE, P, DEFER, OCC, FULL, WGT, PL, false>(a, (int)(it - off[c]));
  }
}

// Register budget per configuration (512 per lane at one wavefront per SIMD):
// ring of P tiles, the query views, one or two accumulator sets.  Few queries
// (memory-bound): a ring of up to four tiles (deeper rings measured no faster)
// and the deferred filter.  Many queries (matrix-core bound, NB = 4): the views
// take most registers, so the ring is shallow and the filter is not deferred.
// P is also bounded by the 63 loads the vector memory counter tracks.
template <int FMT, int KS, int NB>
struct ScanCfg {
  static constexpr int per_tile = KS * (int)sizeof(typename MfmaOp<FMT>::S) / 4;
  static constexpr int views = NB * KS * (int)sizeof(typename MfmaOp<FMT>::T) / 4;
  static constexpr bool defer = NB < 4;
  static constexpr int budget = 440 - views - (defer ? 2 : 1) * NB * 16 - 48;
  static constexpr int p0 = budget / per_tile;
  static constexpr int pv = 63 / KS + 1;
  static constexpr int p1 = p0 < pv ? p0 : pv;
  static constexpr int P = p1 < 2 ? 2 : (p1 > 4 ? 4 : p1);
};

// launch shape of S2/S3 for one scan
struct Shape {
  bool shared;  // the four wavefronts of a workgroup share one query block
  int nb;       // 32-query blocks per wavefront
  int R;        // row ranges per query block
  int64_t nqb;  // query blocks
  int grid;     // workgroups
  int xcd_map;
};

// Query blocks that share rows (SHARED = false) take the tiles through an LDS
// ring shared by the workgroup: one fetch per workgroup instead of one per
// wavefront.  Tiles above 16 KiB (FP32 rows) keep per-wavefront register rings.
template <int FMT, int KS>
struct RingCfg {
  static constexpr int TB = KS * 64 * MfmaOp<FMT>::EPL * MfmaOp<FMT>::EB;
  static constexpr bool ok = FMT != GV_FP32 && TB <= 16384;
  static constexpr int PL = TB <= 10240 ? 5 : 4;
};

// Compile-time configuration of one k_scan instantiation, shared by the launch
// and by the host-side plan checks (scan_limits).  With two query blocks per
// wavefront on the LDS ring, two workgroups share a CU (two wavefronts per SIMD,
// 256 registers each): one wavefront's filter, barrier and LDS waits overlap the
// other's matrix-core chain.  Two such workgroups must fit the LDS: the ring is
// five tiles deep up to 10 KiB tiles (with a 768-key compaction staging at 10
// KiB, 1024 below), four at 12 KiB, three at 16 KiB (768 keys at both).
template <int FMT, int KS, int NB, bool SHARED>
struct KernelCfg {
  using Cfg = ScanCfg<FMT, KS, NB>;
  static constexpr bool W = !SHARED && RingCfg<FMT, KS>::ok;  // workgroup-shared LDS tile ring
  static constexpr int OC = (W && NB == 2) ? 2 : 1;             // workgroups per CU
  static constexpr int PL = W ? (OC == 2 ? ring_tiles_two_per_cu<FMT, KS, NB>() : RingCfg<FMT, KS>::PL) : 1;
  static constexpr bool DEF = W || Cfg::defer;
  static constexpr int P = Cfg::P;
  // tiles between two overflow checks of a list (the kernel's unrolled steps)
  static constexpr int U = W ? 2 : (DEF ? 2 * P : P);
  // keys a compaction can stage in the wavefront's LDS
  static constexpr int CAPL = staging_keys<FMT, KS, NB, OC, W, PL>();
};

template <int FMT, int KS, int NB, bool SHARED, int MODE>
void launch_one(const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  using K = KernelCfg<FMT, KS, NB, SHARED>;
  if (MODE == kFilter && args.stride == 1 && args.repair)
    hipLaunchKernelGGL((k_scan_repair<FMT, KS, NB, SHARED, K::P, K::DEF, K::OC, K::W, K::PL>), dim3(sh.grid),
                       dim3(256), 0, st, args);
  else if (MODE == kFilter && args.stride == 1)
    hipLaunchKernelGGL((k_scan<FMT, KS, NB, SHARED, MODE, K::P, K::DEF, K::OC, true, K::W, K::PL>), dim3(sh.grid),
                       dim3(256), 0, st, args);
  else
    hipLaunchKernelGGL((k_scan<FMT, KS, NB, SHARED, MODE, K::P, K::DEF, K::OC, false, K::W, K::PL>), dim3(sh.grid),
                       dim3(256), 0, st, args);
}

// The lazy variant (Algorithm 3): FP16 storage, one shared block of up to 32
// queries, padded length 160.
template <int MODE>
void launch_lazy(const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  using K = KernelCfg<GV_FP16, 10, 1, true>;
  if (MODE == kFilter && args.stride == 1 && args.repair)
    hipLaunchKernelGGL((k_scan_repair<GV_FP16, 10, 1, true, K::P, K::DEF, K::OC, K::W, K::PL, true>), dim3(sh.grid),
                       dim3(256), 0, st, args);
  else if (MODE == kFilter && args.stride == 1)
    hipLaunchKernelGGL((k_scan<GV_FP16, 10, 1, true, MODE, K::P, K::DEF, K::OC, true, K::W, K::PL, true>),
                       dim3(sh.grid), dim3(256), 0, st, args);
  else
    hipLaunchKernelGGL((k_scan<GV_FP16, 10, 1, true, MODE, K::P, K::DEF, K::OC, false, K::W, K::PL, true>),
                       dim3(sh.grid), dim3(256), 0, st, args);
}

// The instantiation launch_score picks for a shape, described on the host.
struct ScanLimits {
  int nb = 0, U = 0, CAPL = 0, P = 0, PL = 0, occupancy = 0;
  bool ring = false, defer = false;
};

template <int FMT, int KS, int NB, bool SHARED>
ScanLimits limits_of() {
  using K = KernelCfg<FMT, KS, NB, SHARED>;
  ScanLimits l;
  l.nb = NB; l.U = K::U; l.CAPL = K::CAPL; l.P = K::P; l.PL = K::PL; l.occupancy = K::OC;
  l.ring = K::W; l.defer = K::DEF;
  return l;
}

// mirrors launch_score's choice of NB and SHARED
template <int FMT, int KS>
ScanLimits limits_for_shape(const Shape& sh) {
  if constexpr (FMT == GV_FP32) {
    return sh.shared ? limits_of<FMT, KS, 1, true>() : limits_of<FMT, KS, 1, false>();
  } else {
    if (sh.shared && sh.nb == 1) return limits_of<FMT, KS, 1, true>();
    if (sh.shared) return limits_of<FMT, KS, 2, true>();
    if constexpr (KS <= 10) {
      if (sh.nb == 4) return limits_of<FMT, KS, 4, false>();
    }
    return limits_of<FMT, KS, 2, false>();
  }
}

template <int FMT, int KS, int MODE>
void launch_score(const Shape& sh, const ScoreArgs& args, hipStream_t st) {
  if constexpr (FMT == GV_FP32) {
    if (sh.shared) launch_one<FMT, KS, 1, true, MODE>(sh, args, st);
    else launch_one<FMT, KS, 1, false, MODE>(sh, args, st);
  } else {
    if (sh.shared && sh.nb == 1) launch_one<FMT, KS, 1, true, MODE>(sh, args, st);
    else if (sh.shared) launch_one<FMT, KS, 2, true, MODE>(sh, args, st);
    else if constexpr (KS <= 10) {
      if (sh.nb == 4) launch_one<FMT, KS, 4, false, MODE>(sh, args, st);
      else launch_one<FMT, KS, 2, false, MODE>(sh, args, st);
    } else {
      launch_one<FMT, KS, 2, false, MODE>(sh, args, st);
    }
  }
}

template <int FMT, int KS, int NB, bool SHARED>
void launch_queue_one(int grid, const ScoreArgs* args, const int64_t* off, int ncoll, int* head, hipStream_t st) {
  using K = KernelCfg<FMT, KS, NB, SHARED>;
  hipLaunchKernelGGL((k_scan_queue<FMT, KS, NB, SHARED, kFilter, K::P, K::DEF, K::OC, true, K::W, K::PL>),
                     dim3(grid), dim3(256), 0, st, args, off, ncoll, head);
}

// the full-scan instantiation launch_score picks for a shape, as a queue kernel
template <int FMT, int KS>
void launch_queue(const Shape& sh, int grid, const ScoreArgs* args, const int64_t* off, int ncoll, int* head,
                  hipStream_t st) {
  if constexpr (FMT == GV_FP32) {
    if (sh.shared) launch_queue_one<FMT, KS, 1, true>(grid, args, off, ncoll, head, st);
    else launch_queue_one<FMT, KS, 1, false>(grid, args, off, ncoll, head, st);
  } else {
    if (sh.shared && sh.nb == 1) launch_queue_one<FMT, KS, 1, true>(grid, args, off, ncoll, head, st);
    else if (sh.shared) launch_queue_one<FMT, KS, 2, true>(grid, args, off, ncoll, head, st);
    else if constexpr (KS <= 10) {
      if (sh.nb == 4) launch_queue_one<FMT, KS, 4, false>(grid, args, off, ncoll, head, st);
      else launch_queue_one<FMT, KS, 2, false>(grid, args, off, ncoll, head, st);
    } else {
      launch_queue_one<FMT, KS, 2, false>(grid, args, off, ncoll, head, st);
    }
  }
}

template <int FMT>
gv_status dispatch_queue_ks(int dp, const Shape& sh, int grid, const ScoreArgs* args, const int64_t* off, int ncoll,
                            int* head, hipStream_t st) {
  constexpr int km = MfmaOp<FMT>::KM;
  switch (dp / km) {
    case 32 / km: launch_queue<FMT, 32 / km>(sh, grid, args, off, ncoll, head, st); break;
    case 64 / km: launch_queue<FMT, 64 / km>(sh, grid, args, off, ncoll, head, st); break;
    case 128 / km: launch_queue<FMT, 128 / km>(sh, grid, args, off, ncoll, head, st); break;
    case 160 / km: launch_queue<FMT, 160 / km>(sh, grid, args, off, ncoll, head, st); break;
    case 192 / km: launch_queue<FMT, 192 / km>(sh, grid, args, off, ncoll, head, st); break;
    case 256 / km: launch_queue<FMT, 256 / km>(sh, grid, args, off, ncoll, head, st); break;
    default:
      set_error("reduced dimension above 256 is not supported by the scoring kernel");
      return GV_EUNSUPPORTED;
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
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

// per-format entry points (scan_fp32.hip, scan_fp16.hip, ...)
template <int FMT, int MODE>
gv_status dispatch_scan(int dp, const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st);
// the lazy variant (scan_fp16.hip)
template <int MODE>
gv_status dispatch_scan_lazy(const scan::Shape& sh, const scan::ScoreArgs& args, hipStream_t st);
// the persistent full scan over several searches (grid workgroups pull the
// pieces of the searches' argument blocks args[0, ncoll) from the queue *head)
template <int FMT>
gv_status dispatch_scan_queue(int dp, const scan::Shape& sh, int grid, const scan::ScoreArgs* args,
                              const int64_t* off, int ncoll, int* head, hipStream_t st);

}  // namespace gv
