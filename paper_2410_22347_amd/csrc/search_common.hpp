// Device building blocks of the search path: matrix-core operand types per
// storage format, and the workgroup-level selection of the kappa-th largest
// 64-bit key used by the top-kappa stages.
#pragma once

#include "common.hpp"

namespace gv {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Per-format operand of v_mfma_f32_32x32x{16,2}: each lane holds EPL
// consecutive k of one row (A) or one query (B); lanes 32..63 hold the next EPL.
// S is the stored type loaded from memory, T the matrix-core operand, cvt the
// (exact) conversion and kScale the factor cvt applies to each stored value.
// The query view (B) is stored as QS, QEB bytes per element, and reaches the
// matrix core unchanged.
//
// FP8-E4M3 storage is widened to FP16 in registers: placing the sign in bit 15
// and the exponent and fraction fields in bits 7..13 gives, for every finite
// E4M3 code (normal or subnormal), exactly the E4M3 value times 2^-8.  The
// FP16 matrix core then multiplies it with the FP16 query view: the products
// (11 x 4 significant bits) are exact, accumulated in FP32.
template <int FMT>
struct MfmaOp;

template <>
struct MfmaOp<GV_FP32> {
  using S = float;
  using T = float;
  using QS = float;
  static constexpr int KM = 2, EPL = 1, EB = 4, QEB = 4;
  static constexpr float kScale = 1.0f;
  __device__ static inline T cvt(S v) { return v; }
  __device__ static inline f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};
template <>
struct MfmaOp<GV_FP16> {
  using S = f16x8;
  using T = f16x8;
  using QS = f16x8;
  static constexpr int KM = 16, EPL = 8, EB = 2, QEB = 2;
  static constexpr float kScale = 1.0f;
  __device__ static inline T cvt(S v) { return v; }
  __device__ static inline f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};
template <>
struct MfmaOp<GV_BF16> {
  using S = bf16x8;
  using T = bf16x8;
  using QS = bf16x8;
  static constexpr int KM = 16, EPL = 8, EB = 2, QEB = 2;
  static constexpr float kScale = 1.0f;
  __device__ static inline T cvt(S v) { return v; }
  __device__ static inline f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// two E4M3 bytes (bits 0..7 and 8..15 of w) -> two FP16 lanes, value * 2^-8
__device__ inline uint32_t e4m3x2_to_f16x2(uint32_t w) {
  const uint32_t e = ((w << 8) & 0x0000FF00u) | ((w << 16) & 0xFF000000u);
  return (e & 0x80008000u) | ((e >> 1) & 0x3F803F80u);
}

template <>
struct MfmaOp<GV_FP8_E4M3> {
  using S = u32x2;
  using T = f16x8;
  using QS = f16x8;
  static constexpr int KM = 16, EPL = 8, EB = 1, QEB = 2;
  static constexpr float kScale = 0.00390625f;  // 2^-8
  __device__ static inline T cvt(S v) {
    u32x4 h;
    h[0] = e4m3x2_to_f16x2(v[0]);
    h[1] = e4m3x2_to_f16x2(v[0] >> 16);
    h[2] = e4m3x2_to_f16x2(v[1]);
    h[3] = e4m3x2_to_f16x2(v[1] >> 16);
    return __builtin_bit_cast(T, h);
  }
  __device__ static inline f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};

template <typename T>
__device__ inline T zero_op() {
  T z;
  __builtin_memset(&z, 0, sizeof(T));
  return z;
}

// Scratch for block_kth: 256-bin histogram plus broadcast slots.
struct SelectSmem {
  uint32_t hist[256];
  uint64_t prefix;
  uint32_t need;
  uint32_t done;
  uint32_t count;
};

// kappa-th largest of the distinct keys keys[0..cnt) (1 <= kappa <= cnt), by an
// MSB-first radix select with 8-bit digits, for a 256-thread workgroup.
// Returns T such that exactly kappa keys are >= T.  Every thread must call it.
template <typename KeyPtr>
__device__ uint64_t block_kth(KeyPtr keys, int cnt, int kappa, SelectSmem& sm) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    sm.prefix = 0;
    sm.need = (uint32_t)kappa;
    sm.done = 0;
  }
  uint64_t mask = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    sm.hist[tid] = 0;
    __syncthreads();
    const uint64_t prefix = sm.prefix;
    for (int i = tid; i < cnt; i += 256) {
      uint64_t k = keys[i];
      if ((k & mask) == prefix) atomicAdd(&sm.hist[(k >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      // suffix sums over bins (from the top): lane l owns bins 4l..4l+3
      uint32_t h0 = sm.hist[4 * tid], h1 = sm.hist[4 * tid + 1], h2 = sm.hist[4 * tid + 2], h3 = sm.hist[4 * tid + 3];
      uint32_t local = h0 + h1 + h2 + h3;
      uint32_t incl = local;  // sum over lanes >= tid
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t v = __shfl_down(incl, o);
        if (tid + o < 64) incl += v;
      }
      uint32_t above = incl - local;  // keys in bins above this lane's four
      const uint32_t need = sm.need;
      // find bin b (descending within the lane) with above(b) < need <= above(b) + hist[b]
      uint32_t hb[4] = {h0, h1, h2, h3};
      uint32_t a = above;
      for (int j = 3; j >= 0; --j) {
        if (a < need && need <= a + hb[j]) {
          const uint64_t digit = (uint64_t)(4 * tid + j);
          sm.prefix = prefix | (digit << shift);
          sm.need = need - a;
          if (hb[j] == need - a) sm.done = 1;  // every key of this bin is in
        }
        a += hb[j];
      }
    }
    __syncthreads();
    mask |= (uint64_t)255 << shift;
    if (sm.done) break;
  }
  uint64_t t = sm.prefix;
  __syncthreads();
  return t;
}

}  // namespace gv
