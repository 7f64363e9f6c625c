// The inner-product approximation loss and its gradient with respect to the
// per-cluster projections (Problem 3 of the paper, summed over clusters, in the
// second-moment form that Section 3 derives from it), and the statistics it
// needs.
//
// For cluster c, with sums K_Q = sum_q q q^T and K_c = sum_{x in X_c} x x^T,
//   L_c = sum_q sum_{x in X_c} (<A_c q, B_c x> - <q, x>)^2 = <K_Q M_c K_c, M_c>_F,
//   M_c = A_c^T B_c - I.
// Expanding M_c keeps every product at most d x D x D:
//   G1 = A_c K_Q, G2 = B_c K_c (d x D), H_A = G1 A_c^T, H_B = G2 B_c^T (d x d),
//   L_c = <H_A, H_B> - 2 <G1, G2> + <K_Q, K_c>,
//   dL_c/dA_c = 2 (H_B A_c - G2) K_Q,  dL_c/dB_c = 2 (H_A B_c - G1) K_c,
// the same values as 2 B_c K_c M_c^T K_Q and 2 A_c K_Q M_c K_c.  The loss is
// divided by the number of pairs N.  Everything runs in FP64 on the matrix core
// (batched over clusters); the gradients are rounded to FP32 once at the end.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

constexpr int kDotBlocks = 64;  // partial sums per cluster and term

// part[z * kDotBlocks + b] = sum over this block's share of x[z] . y[z]
__global__ __launch_bounds__(256) void k_dot_parts(const double* __restrict__ x, int64_t xs,
                                                   const double* __restrict__ y, int64_t ys, int64_t len,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  const int z = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  const double* xp = x + (int64_t)z * xs;
  const double* yp = y + (int64_t)z * ys;
  const int64_t chunk = (len + kDotBlocks - 1) / kDotBlocks;
  const int64_t i0 = (int64_t)b * chunk, i1 = std::min<int64_t>(len, i0 + chunk);
  double s = 0.0;
  for (int64_t i = i0 + tid; i < i1; i += 256) s += xp[i] * yp[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) part[(int64_t)z * kDotBlocks + b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss = sum_c (t1 - 2 t2 + t3) / N, summed in a fixed order
__global__ void k_loss_combine(const double* __restrict__ p1, const double* __restrict__ p2,
                               const double* __restrict__ p3, int C, double inv_n, double* __restrict__ loss) {
  __shared__ double red[64];
  const int tid = threadIdx.x;  // 64 threads
  double s = 0.0;
  for (int c = 0; c < C; ++c) {
    const int64_t o = (int64_t)c * kDotBlocks + tid;
    s += p1[o] - 2.0 * p2[o] + p3[o];
  }
  red[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < 64; ++i) t += red[i];
    *loss = t * inv_n;
  }
}

__global__ void k_negate(const double* __restrict__ x, double* __restrict__ y, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = -x[i];
}

__global__ void k_fill_f64(double* __restrict__ y, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

template <typename T>
struct Scratch {
  T* p = nullptr;
  hipStream_t st;
  explicit Scratch(hipStream_t s) : st(s) {}
  gv_status alloc(size_t count) {
    if (dev_malloc_async((void**)&p, sizeof(T) * std::max<size_t>(count, 1), st) != hipSuccess) {
      set_error("loss scratch allocation failed");
      return GV_ENOMEM;
    }
    return GV_OK;
  }
  ~Scratch() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

}  // namespace

gv_status loss_grad_impl(int C, int d, int D, const float* A, const float* B, const double* KQ, const double* KX,
                         double n_pairs, double* loss, float* dA, float* dB, hipStream_t st) {
  const int64_t dD = (int64_t)d * D, dd = (int64_t)d * d, DD = (int64_t)D * D;
  Scratch<double> G1(st), G2(st), HA(st), HB(st), E(st), parts(st);
  GV_TRY(G1.alloc(C * dD));
  GV_TRY(G2.alloc(C * dD));
  GV_TRY(HA.alloc(C * dd));
  GV_TRY(HB.alloc(C * dd));
  GV_TRY(parts.alloc(3 * (size_t)C * kDotBlocks));

  using L = Layout;
  const GemmOperand<float> a_rows{A, D, nullptr, L::RowMajor, dD}, b_rows{B, D, nullptr, L::RowMajor, dD};
  const GemmOperand<float> a_kmaj{A, D, nullptr, L::KMajor, dD}, b_kmaj{B, D, nullptr, L::KMajor, dD};
  const GemmOperand<double> kq{KQ, D, nullptr, L::RowMajor, 0}, kx{KX, D, nullptr, L::RowMajor, DD};
  // G1 = A K_Q, G2 = B K_c  (K symmetric: b(j, k) = K[j][k] = K[k][j])
  GV_TRY(gemm_f64<float, double>(d, D, D, a_rows, kq, Epi::StoreF64, GemmOut{G1.p, D, 0, 0, nullptr, dD}, st, C));
  GV_TRY(gemm_f64<float, double>(d, D, D, b_rows, kx, Epi::StoreF64, GemmOut{G2.p, D, 0, 0, nullptr, dD}, st, C));
  // H_A = G1 A^T, H_B = G2 B^T
  const GemmOperand<double> g1{G1.p, D, nullptr, L::RowMajor, dD}, g2{G2.p, D, nullptr, L::RowMajor, dD};
  GV_TRY(gemm_f64<double, float>(d, d, D, g1, a_rows, Epi::StoreF64, GemmOut{HA.p, d, 0, 0, nullptr, dd}, st, C));
  GV_TRY(gemm_f64<double, float>(d, d, D, g2, b_rows, Epi::StoreF64, GemmOut{HB.p, d, 0, 0, nullptr, dd}, st, C));

  // loss terms: <H_A, H_B>, <G1, G2>, <K_Q, K_c>
  double* p1 = parts.p;
  double* p2 = parts.p + (size_t)C * kDotBlocks;
  double* p3 = parts.p + 2 * (size_t)C * kDotBlocks;
  const dim3 dgrid(kDotBlocks, C);
  hipLaunchKernelGGL(k_dot_parts, dgrid, dim3(256), 0, st, HA.p, dd, HB.p, dd, dd, p1);
  hipLaunchKernelGGL(k_dot_parts, dgrid, dim3(256), 0, st, G1.p, dD, G2.p, dD, dD, p2);
  hipLaunchKernelGGL(k_dot_parts, dgrid, dim3(256), 0, st, KQ, (int64_t)0, KX, DD, DD, p3);
  hipLaunchKernelGGL(k_loss_combine, dim3(1), dim3(64), 0, st, p1, p2, p3, C, 1.0 / n_pairs, loss);
  GV_HIP(hipGetLastError());
  if (!dA && !dB) return GV_OK;

  GV_TRY(E.alloc(C * dD));
  const unsigned eg = (unsigned)std::min<int64_t>(4096, (C * dD + 255) / 256);
  const GemmOperand<double> ha{HA.p, d, nullptr, L::RowMajor, dd}, hb{HB.p, d, nullptr, L::RowMajor, dd};
  const GemmOperand<double> e{E.p, D, nullptr, L::RowMajor, dD};
  if (dA) {
    // E = H_B A - G2, dA = (2/N) E K_Q
    hipLaunchKernelGGL(k_negate, dim3(eg), dim3(256), 0, st, G2.p, E.p, C * dD);
    GV_TRY(gemm_f64<double, float>(d, D, d, hb, a_kmaj, Epi::AddF64, GemmOut{E.p, D, 0, 0, nullptr, dD}, st, C));
    GV_TRY(gemm_f64<double, double>(d, D, D, e, kq, Epi::StoreF32, GemmOut{dA, D, 0, 0, nullptr, dD, 2.0 / n_pairs},
                                    st, C));
  }
  if (dB) {
    // E = H_A B - G1, dB = (2/N) E K_c
    hipLaunchKernelGGL(k_negate, dim3(eg), dim3(256), 0, st, G1.p, E.p, C * dD);
    GV_TRY(gemm_f64<double, float>(d, D, d, ha, b_kmaj, Epi::AddF64, GemmOut{E.p, D, 0, 0, nullptr, dD}, st, C));
    GV_TRY(gemm_f64<double, double>(d, D, D, e, kx, Epi::StoreF32, GemmOut{dB, D, 0, 0, nullptr, dD, 2.0 / n_pairs},
                                    st, C));
  }
  GV_HIP(hipGetLastError());
  return GV_OK;
}

// K[c] = sum over the rows v of V with tag c of v v^T (FP64 accumulation of
// exact FP32 products), for c < C; all rows belong to cluster 0 without tags.
// sign 0 overwrites K; +1 / -1 adds / subtracts the sums (streaming updates).
gv_status moments_impl(const float* V, int64_t n, int D, const uint8_t* tags, int C, double* K, hipStream_t st,
                       int sign) {
  const int64_t DD = (int64_t)D * D;
  if (sign == 0) {
    const unsigned fg = (unsigned)std::min<int64_t>(4096, (C * DD + 255) / 256);
    hipLaunchKernelGGL(k_fill_f64, dim3(fg), dim3(256), 0, st, K, C * DD, 0.0);
    GV_HIP(hipGetLastError());
  }
  const double alpha = sign < 0 ? -1.0 : 1.0;
  if (n == 0) return GV_OK;
  if (!tags) {
    const GemmOperand<float> v{V, D, nullptr, Layout::KMajor};
    return gemm_f64<float, float>(D, D, n, v, v, Epi::AddF64, GemmOut{K, D, 0, 0, nullptr, 0, alpha}, st);
  }
  // group the rows by tag on the host (statistics are a one-off)
  std::vector<uint8_t> h_tags(n);
  GV_HIP(hipMemcpyAsync(h_tags.data(), tags, n, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> cnt(C + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (h_tags[i] >= C) {
      set_error("gv_moments: tag out of range");
      return GV_EINVAL;
    }
    ++cnt[h_tags[i] + 1];
  }
  for (int c = 0; c < C; ++c) cnt[c + 1] += cnt[c];
  std::vector<int64_t> perm(n), pos(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i) perm[pos[h_tags[i]]++] = i;
  Scratch<int64_t> d_perm(st);
  GV_TRY(d_perm.alloc(n));
  GV_HIP(hipMemcpyAsync(d_perm.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
  for (int c = 0; c < C; ++c) {
    const int64_t nc = cnt[c + 1] - cnt[c];
    if (nc == 0) continue;
    const GemmOperand<float> v{V, D, d_perm.p + cnt[c], Layout::KMajor};
    GV_TRY(gemm_f64<float, float>(D, D, nc, v, v, Epi::AddF64, GemmOut{K + DD * c, D, 0, 0, nullptr, 0, alpha}, st));
  }
  GV_HIP(hipStreamSynchronize(st));  // the host permutation ends with this call
  return GV_OK;
}

}  // namespace gv
