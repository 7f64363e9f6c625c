// FP64 matrix-core GEMM for the fit, encode and query-projection stages.
//
// C(i, j) = sum_k a(i, k) * b(j, k), accumulated in FP64 with
// v_mfma_f64_16x16x4f64.  Operands may be FP32 (converted exactly to FP64 on
// load) or FP64, stored row-major along k ("RowMajor": a(i, k) = p[i][k]) or
// along the output index ("KMajor": a(i, k) = p[k][i]), with an optional row
// gather.  This one kernel serves the k-means assignment dots, the per-cluster
// second moments (sum over rows of x x^T), the reduced vectors B_c x and the
// eager query views A_c q.
//
// Tiling: a 256-thread workgroup owns a 64 x 64 output tile; its four
// wavefronts each own a 32 x 32 quarter.  K advances in steps of 32 through LDS,
// stored k-major so every MFMA operand read is a contiguous 16-element row.
// The next step's operands are loaded into registers while the matrix core
// works on the current one.
#include "common.hpp"

namespace gv {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TK = 32;

template <typename T>
__device__ inline double ld_elem(const T* p, int64_t idx) {
  return (double)p[idx];
}

// Tile shapes: a 256-thread workgroup owns a TM x TN output tile, each of its
// four wavefronts a (TM / 2) x (TN / 2) quarter of (TM / 32) x (TN / 32) blocks
// of 16 x 16.
template <int TM_, int TN_>
struct Tile {
  static constexpr int TM = TM_, TN = TN_, LDSP = (TM > TN ? TM : TN) + 2;
  static constexpr int SA = TK * TM / 256, SB = TK * TN / 256;  // slab elements per thread
  static constexpr int BX = TM / 32, BY = TN / 32;             // 16 x 16 blocks per wavefront
};

// A TK x W slab of an operand into registers (RowMajor: thread -> row i0 +
// tid / (TK / SE), k0 + SE * (tid % (TK / SE)) ..; KMajor: thread -> k0 + tid /
// (W / SE), i0 + SE * (tid % (W / SE)) ..), zero outside the operand.
template <int W, int SE, typename T>
__device__ inline void load_slab(double (&r)[SE], GemmOperand<T> op, int64_t i0, int64_t k0, int64_t M, int64_t K,
                                 int tid) {
  if (op.layout == Layout::RowMajor) {
    constexpr int PR = TK / SE;  // threads per row
    const int rr = tid / PR, kq = (tid % PR) * SE;
    const int64_t i = i0 + rr;
    const int64_t row = (i < M) ? (op.gather ? op.gather[i] : i) : 0;
#pragma unroll
    for (int e = 0; e < SE; ++e) {
      const int64_t k = k0 + kq + e;
      r[e] = (i < M && k < K) ? ld_elem(op.p, row * op.ld + k) : 0.0;
    }
  } else {
    constexpr int PK = W / SE;  // threads per k
    const int kr = tid / PK, iq = (tid % PK) * SE;
    const int64_t k = k0 + kr;
    const int64_t row = (k < K) ? (op.gather ? op.gather[k] : k) : 0;
#pragma unroll
    for (int e = 0; e < SE; ++e) {
      const int64_t i = i0 + iq + e;
      r[e] = (i < M && k < K) ? ld_elem(op.p, row * op.ld + i) : 0.0;
    }
  }
}

// the registers of load_slab into the k-major LDS slab s[k][i]
template <int W, int SE, int LDSP>
__device__ inline void store_slab(double (*s)[LDSP], const double (&r)[SE], Layout layout, int tid) {
  if (layout == Layout::RowMajor) {
    constexpr int PR = TK / SE;
    const int rr = tid / PR, kq = (tid % PR) * SE;
#pragma unroll
    for (int e = 0; e < SE; ++e) s[kq + e][rr] = r[e];
  } else {
    constexpr int PK = W / SE;
    const int kr = tid / PK, iq = (tid % PK) * SE;
#pragma unroll
    for (int e = 0; e < SE; ++e) s[kr][iq + e] = r[e];
  }
}

template <typename TA, typename TB, Epi EPI, typename TL>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a,
                                                  GemmOperand<TB> b, GemmOut out) {
  constexpr int TM = TL::TM, TN = TL::TN, LDSP = TL::LDSP, SA = TL::SA, SB = TL::SB, BX = TL::BX, BY = TL::BY;
  static_assert(TK % SA == 0 && TK % SB == 0 && TM % SA == 0 && TN % SB == 0, "slab split");
  __shared__ double As[TK][LDSP];
  __shared__ double Bs[TK][LDSP];
  a.p += (int64_t)blockIdx.z * a.bstride;
  b.p += (int64_t)blockIdx.z * b.bstride;
  const int64_t zo = (int64_t)blockIdx.z * out.bstride;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * TM, j0 = (int64_t)blockIdx.y * TN;
  const int wi = (wave >> 1) * (TM / 2), wj = (wave & 1) * (TN / 2);

  d4 acc[BX][BY];
#pragma unroll
  for (int x = 0; x < BX; ++x)
#pragma unroll
    for (int y = 0; y < BY; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[SA], rb[SB];
  load_slab<TM, SA>(ra, a, i0, 0, M, K, tid);
  load_slab<TN, SB>(rb, b, j0, 0, N, K, tid);
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    store_slab<TM, SA, LDSP>(As, ra, a.layout, tid);
    store_slab<TN, SB, LDSP>(Bs, rb, b.layout, tid);
    __syncthreads();
    if (k0 + TK < K) {  // the next step's operands travel while this one is multiplied
      load_slab<TM, SA>(ra, a, i0, k0 + TK, M, K, tid);
      load_slab<TN, SB>(rb, b, j0, k0 + TK, N, K, tid);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      double af[BX], bf[BY];
#pragma unroll
      for (int x = 0; x < BX; ++x) af[x] = As[kr][wi + 16 * x + c];
#pragma unroll
      for (int y = 0; y < BY; ++y) bf[y] = Bs[kr][wj + 16 * y + c];
#pragma unroll
      for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < BY; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }

  // D layout of the 16x16 FP64 block: register r of a lane holds column lane%16,
  // row lane/16 + 4r (the rows of one lane are interleaved, unlike the FP32 forms)
#pragma unroll
  for (int x = 0; x < BX; ++x)
#pragma unroll
    for (int y = 0; y < BY; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t i = i0 + wi + 16 * x + (lane >> 4) + 4 * r;
        int64_t j = j0 + wj + 16 * y + (lane & 15);
        if (i >= M || j >= N) continue;
        const double v = out.alpha * acc[x][y][r];
        if (EPI == Epi::StoreF64) {
          ((double*)out.p + zo)[i * out.ldc + j] = v;
        } else if (EPI == Epi::AddF64) {
          ((double*)out.p + zo)[i * out.ldc + j] += v;
        } else if (EPI == Epi::StoreF32Proj) {
          int64_t c = j / out.cd, jj = j - c * out.cd;
          ((float*)out.p + zo)[i * out.ldc + c * out.cdp + jj] = (float)v;
        } else {
          int64_t row = out.row_map ? out.row_map[i] : i;
          ((float*)out.p + zo)[row * out.ldc + j] = (float)v;
        }
      }
}

template <typename TA, typename TB, typename TL>
void launch(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a, GemmOperand<TB> b, Epi epi, GemmOut out,
            hipStream_t st, dim3 grid) {
  switch (epi) {
    case Epi::StoreF64:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF64, TL>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::AddF64:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::AddF64, TL>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::StoreF32Proj:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF32Proj, TL>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::StoreF32:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF32, TL>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
  }
}

}  // namespace

template <typename TA, typename TB>
gv_status gemm_f64(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a, GemmOperand<TB> b, Epi epi,
                   GemmOut out, hipStream_t st, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return GV_OK;
  // 64 x 64 tiles: 128 x 128 tiles (half the operand traffic per flop) measured
  // slower on the S1 product at m = 4096 (1.08 against 0.91 ms)
  using TL = Tile<64, 64>;
  int64_t gx = (M + TL::TM - 1) / TL::TM, gy = (N + TL::TN - 1) / TL::TN;
  if (gy > 65535 || batch > 65535) {
    set_error("gemm_f64: N or batch too large");
    return GV_EINVAL;
  }
  dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)batch);
  launch<TA, TB, TL>(M, N, K, a, b, epi, out, st, grid);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

template gv_status gemm_f64<double, double>(int64_t, int64_t, int64_t, GemmOperand<double>,
                                            GemmOperand<double>, Epi, GemmOut, hipStream_t, int);
template gv_status gemm_f64<float, double>(int64_t, int64_t, int64_t, GemmOperand<float>,
                                           GemmOperand<double>, Epi, GemmOut, hipStream_t, int);
template gv_status gemm_f64<double, float>(int64_t, int64_t, int64_t, GemmOperand<double>,
                                           GemmOperand<float>, Epi, GemmOut, hipStream_t, int);
template gv_status gemm_f64<float, float>(int64_t, int64_t, int64_t, GemmOperand<float>,
                                          GemmOperand<float>, Epi, GemmOut, hipStream_t, int);

}  // namespace gv
