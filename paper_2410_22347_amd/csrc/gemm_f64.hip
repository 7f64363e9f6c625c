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
// wavefronts each own 32 x 32 (2 x 2 blocks of 16 x 16).  K advances in steps
// of 32 through LDS, stored k-major so every MFMA operand read is a
// contiguous 16-element row.  The next step's operands are loaded into
// registers while the matrix core works on the current one.
#include "common.hpp"

namespace gv {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32, LDSP = TM + 2;
constexpr int SE = TK * TM / 256;  // slab elements per thread

template <typename T>
__device__ inline double ld_elem(const T* p, int64_t idx) {
  return (double)p[idx];
}

// A TK x 64 slab of an operand into registers (RowMajor: thread -> row i0 +
// tid / 4, k0 + SE * (tid % 4) ..; KMajor: thread -> k0 + tid / 8, i0 + SE *
// (tid % 8) ..), zero outside the operand.
template <typename T>
__device__ inline void load_slab(double (&r)[SE], GemmOperand<T> op, int64_t i0, int64_t k0, int64_t M, int64_t K,
                                 int tid) {
  if (op.layout == Layout::RowMajor) {
    const int rr = tid >> 2, kq = (tid & 3) * SE;
    const int64_t i = i0 + rr;
    const int64_t row = (i < M) ? (op.gather ? op.gather[i] : i) : 0;
#pragma unroll
    for (int e = 0; e < SE; ++e) {
      const int64_t k = k0 + kq + e;
      r[e] = (i < M && k < K) ? ld_elem(op.p, row * op.ld + k) : 0.0;
    }
  } else {
    const int kr = tid >> 3, iq = (tid & 7) * SE;
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
__device__ inline void store_slab(double (*s)[LDSP], const double (&r)[SE], Layout layout, int tid) {
  if (layout == Layout::RowMajor) {
    const int rr = tid >> 2, kq = (tid & 3) * SE;
#pragma unroll
    for (int e = 0; e < SE; ++e) s[kq + e][rr] = r[e];
  } else {
    const int kr = tid >> 3, iq = (tid & 7) * SE;
#pragma unroll
    for (int e = 0; e < SE; ++e) s[kr][iq + e] = r[e];
  }
}

template <typename TA, typename TB, Epi EPI>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a,
                                                  GemmOperand<TB> b, GemmOut out) {
  __shared__ double As[TK][LDSP];
  __shared__ double Bs[TK][LDSP];
  a.p += (int64_t)blockIdx.z * a.bstride;
  b.p += (int64_t)blockIdx.z * b.bstride;
  const int64_t zo = (int64_t)blockIdx.z * out.bstride;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * TM, j0 = (int64_t)blockIdx.y * TN;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;

  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[SE], rb[SE];
  load_slab(ra, a, i0, 0, M, K, tid);
  load_slab(rb, b, j0, 0, N, K, tid);
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    store_slab(As, ra, a.layout, tid);
    store_slab(Bs, rb, b.layout, tid);
    __syncthreads();
    if (k0 + TK < K) {  // the next step's operands travel while this one is multiplied
      load_slab(ra, a, i0, k0 + TK, M, K, tid);
      load_slab(rb, b, j0, k0 + TK, N, K, tid);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = As[kr][wi + 16 * x + c];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = Bs[kr][wj + 16 * y + c];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }

  // D layout of the 16x16 FP64 block: register r of a lane holds column lane%16,
  // row lane/16 + 4r (the rows of one lane are interleaved, unlike the FP32 forms)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
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

}  // namespace

template <typename TA, typename TB>
gv_status gemm_f64(int64_t M, int64_t N, int64_t K, GemmOperand<TA> a, GemmOperand<TB> b, Epi epi,
                   GemmOut out, hipStream_t st, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return GV_OK;
  int64_t gx = (M + TM - 1) / TM, gy = (N + TN - 1) / TN;
  if (gy > 65535 || batch > 65535) {
    set_error("gemm_f64: N or batch too large");
    return GV_EINVAL;
  }
  dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)batch);
  switch (epi) {
    case Epi::StoreF64:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF64>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::AddF64:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::AddF64>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::StoreF32Proj:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF32Proj>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
    case Epi::StoreF32:
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi::StoreF32>), grid, dim3(256), 0, st, M, N, K, a, b, out);
      break;
  }
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
