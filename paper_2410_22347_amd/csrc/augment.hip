// Euclidean distance through inner products (the paper's appendix on adapting
// other similarities): one appended coordinate per vector,
//   database  x^ = [x, -||x||^2 / 2],   queries  q^ = [q, 1],
// so <q^, x^> = -||q - x||^2 / 2 + ||q||^2 / 2 and the inner-product search on
// the augmented vectors returns the Euclidean nearest neighbours.
#include "common.hpp"

namespace gv {
namespace {

// One wavefront per row: the D values copied, then the appended one (FP64 sum
// of the exact squares, rounded once to FP32, for the database; 1 for queries).
__global__ __launch_bounds__(256) void k_augment(const float* __restrict__ V, int64_t n, int D, int database,
                                                 float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* v = V + row * D;
  float* o = out + row * (int64_t)(D + 1);
  double sq = 0.0;
  for (int j = lane; j < D; j += 64) {
    const float x = v[j];
    o[j] = x;
    sq += (double)x * (double)x;
  }
  for (int s = 32; s > 0; s >>= 1) sq += __shfl_xor(sq, s);
  if (lane == 0) o[D] = database ? (float)(-0.5 * sq) : 1.0f;
}

}  // namespace

gv_status augment_impl(const float* V, int64_t n, int D, int database, float* out, hipStream_t st) {
  if (n == 0) return GV_OK;
  hipLaunchKernelGGL(k_augment, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, V, n, D, database, out);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

}  // namespace gv
