// GleanVec learning (Algorithm 5 of the paper) on the GPU, in FP64.
//
//   landmarks   spherical k-means (Appendix A) on a uniform sample of at most
//               1e5 normalised learn vectors: k-means++ seeding with the squared
//               chord distance 2 - 2 <x~, mu>, then Lloyd steps (arg-max
//               assignment, normalised cluster sums) until no assignment changes;
//   partition   X_c = learn vectors whose arg-max landmark is c (Eq. 9);
//   statistics  K_Q = mean q q^T and K_{X_c} = sum x x^T (Section 3.2), on the
//               FP64 matrix cores;
//   sphering    W = K_Q^(1/2), W+ (Section 3), P_c = leading eigenvectors of
//               W K_{X_c} W, A_c = P_c W+, B_c = P_c W (Algorithm 2, eigen route).
//
// Random draws come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) in a
// fixed order: the sample (partial Fisher-Yates over the learn rows, sorted),
// then the k-means++ draws.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.hpp"

namespace gv {
namespace {

struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

// RAII device allocation
template <typename T>
struct DevBuf {
  T* p = nullptr;
  gv_status alloc(size_t count) {
    if (count == 0) count = 1;
    hipError_t e = dev_malloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
      return GV_ENOMEM;
    }
    return GV_OK;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// x~_r = x_{idx[r]} / |x_{idx[r]}|  (one wavefront per row; zero rows stay zero)
__global__ void k_normalise_gather(const float* __restrict__ X, int64_t ld, const int64_t* __restrict__ idx,
                                   int64_t rows, int D, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= rows) return;
  const float* x = X + idx[r] * ld;
  double ss = 0.0;
  for (int j = lane; j < D; j += 64) {
    double v = (double)x[j];
    ss += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
  double nrm = sqrt(ss);
  double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int j = lane; j < D; j += 64) out[r * D + j] = nrm > 0.0 ? (double)x[j] / nrm : 0.0;
  (void)inv;
}

// best[i] = max(best[i], <Xt_i, mu>) (or = when init)
__global__ void k_rowdot_max(const double* __restrict__ Xt, int64_t rows, int D, const double* __restrict__ mu,
                             double* __restrict__ best, int init) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= rows) return;
  double s = 0.0;
  for (int j = lane; j < D; j += 64) s += Xt[r * D + j] * mu[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) best[r] = init ? s : fmax(best[r], s);
}

// arg-max over the C columns of each row, lowest index on ties
__global__ void k_argmax(const double* __restrict__ dots, int64_t rows, int C, int32_t* __restrict__ out) {
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
  out[r] = best;
}

// Cluster sums in two deterministic passes.  Pass 1: part[c][k][j] = sum of
// Xt[perm[r]][j] over the k-th run of kSumRun members of cluster c (grouped
// order).  Pass 2: S[c][j] = sum over k of part[c][k][j], in order of k.
constexpr int kSumRun = 256;
__global__ void k_cluster_part_sums(const double* __restrict__ Xt, int D, const int64_t* __restrict__ perm,
                                    const int64_t* __restrict__ off, int runs, double* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.z, k = blockIdx.y;
  if (j >= D) return;
  const int64_t r0 = off[c] + (int64_t)k * kSumRun, r1 = std::min<int64_t>(off[c + 1], r0 + kSumRun);
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += Xt[perm[r] * D + j];
  part[((int64_t)c * runs + k) * D + j] = s;
}
__global__ void k_cluster_sums(const double* __restrict__ part, int D, int runs, double* __restrict__ S) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= D) return;
  double s = 0.0;
  for (int k = 0; k < runs; ++k) s += part[((int64_t)c * runs + k) * D + j];
  S[(int64_t)c * D + j] = s;
}

void counting_sort(const std::vector<int32_t>& a, int C, std::vector<int64_t>& perm, std::vector<int64_t>& off) {
  off.assign(C + 1, 0);
  for (int32_t v : a) off[v + 1]++;
  for (int c = 0; c < C; ++c) off[c + 1] += off[c];
  perm.resize(a.size());
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (size_t i = 0; i < a.size(); ++i) perm[pos[a[i]]++] = (int64_t)i;
}

gv_status assign_rows(const GemmOperand<double>& xt, int64_t rows, const double* mu, int C, int D, double* dots,
                      int32_t* out, hipStream_t st) {
  GemmOperand<double> m{mu, D, nullptr, Layout::RowMajor};
  GV_TRY(gemm_f64<double, double>(rows, C, D, xt, m, Epi::StoreF64, GemmOut{dots, C, 0, 0, nullptr}, st));
  hipLaunchKernelGGL(k_argmax, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, dots, rows, C, out);
  GV_HIP(hipGetLastError());
  return GV_OK;
}

void canonical_signs(double* P, int d, int D) {
  for (int r = 0; r < d; ++r) {
    double* row = P + (size_t)r * D;
    int jm = 0;
    for (int j = 1; j < D; ++j)
      if (std::fabs(row[j]) > std::fabs(row[jm])) jm = j;
    if (row[jm] < 0)
      for (int j = 0; j < D; ++j) row[j] = -row[j];
  }
}

template <typename F>
void parallel_for(int count, F f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max(1u, std::min(hw == 0 ? 4u : hw, 16u));
  nt = std::min(nt, count);
  if (nt <= 1) {
    for (int i = 0; i < count; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int> next{0};
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) f(i);
    });
  for (auto& t : th) t.join();
}

}  // namespace

// Sphering and per-cluster projections from the statistics (Section 3.2,
// Algorithm 2 through eigendecompositions): W, W+ from model->KQ (the mean
// second moment of the queries, host), P_c from W K_c W with K_c = KX_dev
// (device, C x D x D sums; model->KX holds the same on the host), then
// A_c = P_c W+, B_c = P_c W.  A cluster with fewer than d vectors takes the
// projection of the pooled statistics.  mu_dev: the C x D landmarks (device).
gv_status sphere_project(gv_model* model, const double* KX_dev, const std::vector<int64_t>& counts,
                         const double* mu_dev, hipStream_t st) {
  const int C = model->C, d = model->d, D = model->D;
  const size_t DD = (size_t)D * D;
  DevBuf<double> W, Wp, tmp, Y;
  // ------------------------------------------------ sphering: W, W+
  std::vector<double> Aq(model->KQ), lamQ, Uq;
  if (!eigh_desc(D, Aq, lamQ, Uq)) {
    set_error("fit: the eigendecomposition of K_Q did not converge");
    return GV_ENOCONV;
  }
  const double rcond = (double)D * 0x1.0p-52;
  std::vector<double> VS(DD), VSp(DD);
  for (int r = 0; r < D; ++r) {
    double s = std::sqrt(std::max(lamQ[r], 0.0));
    double sp = (lamQ[0] > 0 && lamQ[r] > rcond * lamQ[0]) ? 1.0 / s : 0.0;
    for (int j = 0; j < D; ++j) {
      VS[(size_t)r * D + j] = s * Uq[(size_t)r * D + j];
      VSp[(size_t)r * D + j] = sp * Uq[(size_t)r * D + j];
    }
  }
  GV_TRY(W.alloc(DD));
  GV_TRY(Wp.alloc(DD));
  GV_TRY(tmp.alloc(DD * 3));
  {
    double* d_vs = tmp.p;
    double* d_vsp = tmp.p + DD;
    double* d_u = tmp.p + 2 * DD;
    GV_HIP(hipMemcpyAsync(d_vs, VS.data(), sizeof(double) * DD, hipMemcpyHostToDevice, st));
    GV_HIP(hipMemcpyAsync(d_vsp, VSp.data(), sizeof(double) * DD, hipMemcpyHostToDevice, st));
    GV_HIP(hipMemcpyAsync(d_u, Uq.data(), sizeof(double) * DD, hipMemcpyHostToDevice, st));
    // W(i, j) = sum_r S_r U(i, r) U(j, r), U(i, r) = Vt[r][i]
    GemmOperand<double> a1{d_vs, D, nullptr, Layout::KMajor}, b1{d_u, D, nullptr, Layout::KMajor};
    GV_TRY(gemm_f64<double, double>(D, D, D, a1, b1, Epi::StoreF64, GemmOut{W.p, D, 0, 0, nullptr}, st));
    GemmOperand<double> a2{d_vsp, D, nullptr, Layout::KMajor};
    GV_TRY(gemm_f64<double, double>(D, D, D, a2, b1, Epi::StoreF64, GemmOut{Wp.p, D, 0, 0, nullptr}, st));
    GV_HIP(hipStreamSynchronize(st));
  }

  // ------------------------------------------------ per-cluster projections
  std::vector<uint8_t> fallback(C);
  bool any_fb = false;
  for (int c = 0; c < C; ++c) {
    fallback[c] = counts[c] < d ? 1 : 0;
    any_fb |= fallback[c] != 0;
  }
  const int nY = C + (any_fb ? 1 : 0);
  GV_TRY(Y.alloc(DD * nY));
  DevBuf<double> Kpool;
  if (any_fb) {
    std::vector<double> pool(DD, 0.0);
    for (int c = 0; c < C; ++c)
      for (size_t e = 0; e < DD; ++e) pool[e] += model->KX[DD * c + e];
    GV_TRY(Kpool.alloc(DD));
    GV_HIP(hipMemcpyAsync(Kpool.p, pool.data(), sizeof(double) * DD, hipMemcpyHostToDevice, st));
  }
  GemmOperand<double> w_op{W.p, D, nullptr, Layout::RowMajor};
  for (int c = 0; c < nY; ++c) {
    const double* K = (c < C) ? KX_dev + DD * c : Kpool.p;
    if (c < C && fallback[c]) continue;
    // T = W K  (K symmetric: T(i, j) = sum_k W(i, k) K(j, k)), then Y = T W
    GemmOperand<double> k_op{K, D, nullptr, Layout::RowMajor};
    GV_TRY(gemm_f64<double, double>(D, D, D, w_op, k_op, Epi::StoreF64, GemmOut{tmp.p, D, 0, 0, nullptr}, st));
    GemmOperand<double> t_op{tmp.p, D, nullptr, Layout::RowMajor};
    GV_TRY(gemm_f64<double, double>(D, D, D, t_op, w_op, Epi::StoreF64, GemmOut{Y.p + DD * c, D, 0, 0, nullptr}, st));
  }
  std::vector<double> hY(DD * nY);
  GV_HIP(hipMemcpyAsync(hY.data(), Y.p, sizeof(double) * DD * nY, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));

  std::vector<double> P((size_t)C * d * D), lamc((size_t)C * D);
  std::vector<std::vector<double>> lam_all(nY), P_all(nY);
  std::vector<int> jobs;
  for (int c = 0; c < nY; ++c)
    if (c == C || !fallback[c]) jobs.push_back(c);
  std::vector<uint8_t> converged(nY, 1);
  parallel_for((int)jobs.size(), [&](int ji) {
    int c = jobs[ji];
    std::vector<double> Ysym(DD);
    const double* y = hY.data() + DD * c;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) Ysym[(size_t)i * D + j] = 0.5 * (y[(size_t)i * D + j] + y[(size_t)j * D + i]);
    std::vector<double> lam, Vt;
    converged[c] = eigh_desc(D, Ysym, lam, Vt) ? 1 : 0;
    Vt.resize((size_t)d * D);
    canonical_signs(Vt.data(), d, D);
    lam_all[c] = std::move(lam);
    P_all[c] = std::move(Vt);
  });
  for (int c = 0; c < nY; ++c) {
    if (!converged[c]) {
      set_error("fit: the eigendecomposition of W K_c W did not converge for cluster " + std::to_string(c));
      return GV_ENOCONV;
    }
  }
  for (int c = 0; c < C; ++c) {
    int src = fallback[c] ? C : c;
    std::copy(P_all[src].begin(), P_all[src].end(), P.begin() + (size_t)c * d * D);
    std::copy(lam_all[src].begin(), lam_all[src].end(), lamc.begin() + (size_t)c * D);
  }

  // A = P W+, B = P W (W, W+ symmetric), all clusters in one product each
  DevBuf<double> dP;
  GV_TRY(dP.alloc((size_t)C * d * D));
  GV_HIP(hipMemcpyAsync(dP.p, P.data(), sizeof(double) * C * d * D, hipMemcpyHostToDevice, st));
  GemmOperand<double> p_op{dP.p, D, nullptr, Layout::RowMajor}, wp_op{Wp.p, D, nullptr, Layout::RowMajor};
  GV_TRY(gemm_f64<double, double>((int64_t)C * d, D, D, p_op, wp_op, Epi::StoreF64,
                                  GemmOut{model->A, D, 0, 0, nullptr}, st));
  GV_TRY(gemm_f64<double, double>((int64_t)C * d, D, D, p_op, w_op, Epi::StoreF64,
                                  GemmOut{model->B, D, 0, 0, nullptr}, st));
  GV_HIP(hipMemcpyAsync(model->mu, mu_dev, sizeof(double) * C * D, hipMemcpyDeviceToDevice, st));
  model->W.resize(DD);
  model->Wp.resize(DD);
  GV_HIP(hipMemcpyAsync(model->W.data(), W.p, sizeof(double) * DD, hipMemcpyDeviceToHost, st));
  GV_HIP(hipMemcpyAsync(model->Wp.data(), Wp.p, sizeof(double) * DD, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));

  model->P = std::move(P);
  model->lamQ = lamQ;
  model->lamc = lamc;
  model->counts = counts;
  model->fallback = fallback;
  model->fitted = true;
  return GV_OK;
}

gv_status fit_impl(const float* X, int64_t n, const float* Q, int64_t m, int D, int d, int C, uint64_t seed,
                   const gv_fit_opts* opts, hipStream_t st, gv_model* model) {
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 50;
  const int64_t ks = (opts && opts->kmeans_sample > 0) ? opts->kmeans_sample : 100000;
  const size_t DD = (size_t)D * D;

  // ------------------------------------------------ sample (Appendix A)
  SplitMix64 gen(seed);
  std::vector<int64_t> sample;
  if (ks >= n) {
    sample.resize(n);
    for (int64_t i = 0; i < n; ++i) sample[i] = i;
  } else {
    std::vector<int64_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = 0; i < ks; ++i) {
      int64_t j = i + (int64_t)(gen.next() % (uint64_t)(n - i));
      std::swap(perm[i], perm[j]);
    }
    sample.assign(perm.begin(), perm.begin() + ks);
    std::sort(sample.begin(), sample.end());
  }
  const int64_t ns = (int64_t)sample.size();

  DevBuf<int64_t> d_sample;
  GV_TRY(d_sample.alloc(ns));
  GV_HIP(hipMemcpyAsync(d_sample.p, sample.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, st));
  DevBuf<double> Xt, mu, dots, best, S;
  GV_TRY(Xt.alloc((size_t)ns * D));
  GV_TRY(mu.alloc((size_t)C * D));
  GV_TRY(dots.alloc((size_t)ns * C));
  GV_TRY(best.alloc(ns));
  GV_TRY(S.alloc((size_t)C * D));
  const unsigned rows_grid = (unsigned)((ns + 3) / 4);
  hipLaunchKernelGGL(k_normalise_gather, dim3(rows_grid), dim3(256), 0, st, X, (int64_t)D, d_sample.p, ns, D, Xt.p);
  GV_HIP(hipGetLastError());

  // ------------------------------------------------ seeding
  std::vector<double> h_mu((size_t)C * D);
  if (opts && opts->init_centroids) {
    std::memcpy(h_mu.data(), opts->init_centroids, sizeof(double) * C * D);
    GV_HIP(hipMemcpyAsync(mu.p, h_mu.data(), sizeof(double) * C * D, hipMemcpyHostToDevice, st));
  } else {
    std::vector<double> h_best(ns);
    int64_t first = (int64_t)(gen.next() % (uint64_t)ns);
    GV_HIP(hipMemcpyAsync(mu.p, Xt.p + first * D, sizeof(double) * D, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_rowdot_max, dim3(rows_grid), dim3(256), 0, st, Xt.p, ns, D, mu.p, best.p, 1);
    GV_HIP(hipGetLastError());
    for (int c = 1; c < C; ++c) {
      GV_HIP(hipMemcpyAsync(h_best.data(), best.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
      GV_HIP(hipStreamSynchronize(st));
      double total = 0.0;
      std::vector<double> cum(ns);
      for (int64_t i = 0; i < ns; ++i) {
        double d2 = std::max(0.0, 2.0 - 2.0 * h_best[i]);
        total += d2;
        cum[i] = total;
      }
      double u = gen.uniform();
      int64_t pick;
      if (total > 0) {
        double target = u * total;
        pick = std::upper_bound(cum.begin(), cum.end(), target) - cum.begin();  // first cum > target
        if (pick >= ns) pick = ns - 1;
      } else {
        pick = (int64_t)(u * (double)ns);
      }
      GV_HIP(hipMemcpyAsync(mu.p + (int64_t)c * D, Xt.p + pick * D, sizeof(double) * D, hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_rowdot_max, dim3(rows_grid), dim3(256), 0, st, Xt.p, ns, D, mu.p + (int64_t)c * D,
                         best.p, 0);
      GV_HIP(hipGetLastError());
    }
    GV_HIP(hipMemcpyAsync(h_mu.data(), mu.p, sizeof(double) * C * D, hipMemcpyDeviceToHost, st));
  }

  // ------------------------------------------------ Lloyd steps
  DevBuf<int32_t> d_a;
  GV_TRY(d_a.alloc(ns));
  DevBuf<int64_t> d_perm, d_off;
  GV_TRY(d_perm.alloc(ns));
  GV_TRY(d_off.alloc(C + 1));
  GemmOperand<double> xt_op{Xt.p, D, nullptr, Layout::RowMajor};
  std::vector<int32_t> a(ns), a_new(ns);
  GV_TRY(assign_rows(xt_op, ns, mu.p, C, D, dots.p, d_a.p, st));
  GV_HIP(hipMemcpyAsync(a.data(), d_a.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  int it = 0;
  std::vector<int64_t> perm, off;
  std::vector<double> h_S((size_t)C * D);
  for (it = 1; it <= max_iter; ++it) {
    counting_sort(a, C, perm, off);
    GV_HIP(hipMemcpyAsync(d_perm.p, perm.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, st));
    GV_HIP(hipMemcpyAsync(d_off.p, off.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, st));
    {
      int64_t largest = 0;
      for (int c = 0; c < C; ++c) largest = std::max<int64_t>(largest, off[c + 1] - off[c]);
      const int runs = (int)std::max<int64_t>(1, (largest + kSumRun - 1) / kSumRun);
      DevBuf<double> part;
      GV_TRY(part.alloc((size_t)C * runs * D));
      hipLaunchKernelGGL(k_cluster_part_sums, dim3((D + 127) / 128, runs, C), dim3(128), 0, st, Xt.p, D, d_perm.p,
                         d_off.p, runs, part.p);
      hipLaunchKernelGGL(k_cluster_sums, dim3((D + 127) / 128, C), dim3(128), 0, st, part.p, D, runs, S.p);
      GV_HIP(hipGetLastError());
      GV_HIP(hipStreamSynchronize(st));  // part is freed (synchronously) at the end of this block
    }
    GV_HIP(hipMemcpyAsync(h_S.data(), S.p, sizeof(double) * C * D, hipMemcpyDeviceToHost, st));
    GV_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < C; ++c) {
      if (off[c + 1] == off[c]) continue;  // empty cluster keeps its centre
      double ss = 0.0;
      for (int j = 0; j < D; ++j) ss += h_S[(size_t)c * D + j] * h_S[(size_t)c * D + j];
      double nrm = std::sqrt(ss);
      if (nrm > 0)
        for (int j = 0; j < D; ++j) h_mu[(size_t)c * D + j] = h_S[(size_t)c * D + j] / nrm;
    }
    GV_HIP(hipMemcpyAsync(mu.p, h_mu.data(), sizeof(double) * C * D, hipMemcpyHostToDevice, st));
    GV_TRY(assign_rows(xt_op, ns, mu.p, C, D, dots.p, d_a.p, st));
    GV_HIP(hipMemcpyAsync(a_new.data(), d_a.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
    GV_HIP(hipStreamSynchronize(st));
    if (a_new == a) break;
    a.swap(a_new);
  }
  if (it > max_iter) it = max_iter;

  // ------------------------------------------------ partition of the learn set
  DevBuf<int32_t> d_tags;
  GV_TRY(d_tags.alloc(n));
  {
    const int64_t chunk = std::min<int64_t>(n, 1 << 20);
    DevBuf<double> cd;
    GV_TRY(cd.alloc((size_t)chunk * C));
    for (int64_t s0 = 0; s0 < n; s0 += chunk) {
      int64_t rows = std::min(chunk, n - s0);
      GemmOperand<float> xo{X + s0 * D, D, nullptr, Layout::RowMajor};
      GemmOperand<double> mo{mu.p, D, nullptr, Layout::RowMajor};
      GV_TRY(gemm_f64<float, double>(rows, C, D, xo, mo, Epi::StoreF64, GemmOut{cd.p, C, 0, 0, nullptr}, st));
      hipLaunchKernelGGL(k_argmax, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, cd.p, rows, C,
                         d_tags.p + s0);
      GV_HIP(hipGetLastError());
    }
  }
  std::vector<int32_t> tags(n);
  GV_HIP(hipMemcpyAsync(tags.data(), d_tags.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  GV_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> lperm, loff;
  counting_sort(tags, C, lperm, loff);

  // ------------------------------------------------ statistics (Section 3.2)
  DevBuf<double> KQ, KX;
  GV_TRY(KQ.alloc(DD));
  GV_TRY(KX.alloc(DD * C));
  {
    GemmOperand<float> qo{Q, D, nullptr, Layout::KMajor};
    GV_TRY(gemm_f64<float, float>(D, D, m, qo, qo, Epi::StoreF64, GemmOut{KQ.p, D, 0, 0, nullptr}, st));
    DevBuf<int64_t> d_lperm;
    GV_TRY(d_lperm.alloc(n));
    GV_HIP(hipMemcpyAsync(d_lperm.p, lperm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
    for (int c = 0; c < C; ++c) {
      int64_t nc = loff[c + 1] - loff[c];
      if (nc == 0) {
        GV_HIP(hipMemsetAsync(KX.p + DD * c, 0, sizeof(double) * DD, st));
        continue;
      }
      GemmOperand<float> xo{X, D, d_lperm.p + loff[c], Layout::KMajor};
      GV_TRY(gemm_f64<float, float>(D, D, nc, xo, xo, Epi::StoreF64, GemmOut{KX.p + DD * c, D, 0, 0, nullptr}, st));
    }
    GV_HIP(hipStreamSynchronize(st));
  }
  model->KQ.resize(DD);
  model->KX.resize(DD * C);
  GV_HIP(hipMemcpy(model->KQ.data(), KQ.p, sizeof(double) * DD, hipMemcpyDeviceToHost));
  GV_HIP(hipMemcpy(model->KX.data(), KX.p, sizeof(double) * DD * C, hipMemcpyDeviceToHost));
  for (auto& v : model->KQ) v /= (double)m;

  std::vector<int64_t> counts(C);
  for (int c = 0; c < C; ++c) counts[c] = loff[c + 1] - loff[c];
  GV_TRY(sphere_project(model, KX.p, counts, mu.p, st));
  model->iters = it;
  return GV_OK;
}

// The projections of a model from statistics kept by the caller (streaming
// updates of Section 3: K_Q and K_{X_c} are sums, updated by adding or
// removing outer products, and the projections are recomputed from them).
// mu: host C x D landmarks; KQ: device D x D sum over m_q queries; KX: device
// C x D x D sums; counts: host C vectors behind each K_{X_c}.
gv_status fit_from_stats_impl(const double* mu, const double* KQ, double m_q, const double* KX,
                              const int64_t* counts, hipStream_t st, gv_model* model) {
  const int C = model->C, D = model->D;
  const size_t DD = (size_t)D * D;
  model->KQ.resize(DD);
  model->KX.resize(DD * C);
  GV_HIP(hipMemcpyAsync(model->KQ.data(), KQ, sizeof(double) * DD, hipMemcpyDeviceToHost, st));
  GV_HIP(hipMemcpyAsync(model->KX.data(), KX, sizeof(double) * DD * C, hipMemcpyDeviceToHost, st));
  GV_HIP(hipMemcpyAsync(model->mu, mu, sizeof(double) * C * D, hipMemcpyHostToDevice, st));
  GV_HIP(hipStreamSynchronize(st));
  for (auto& v : model->KQ) v /= m_q;
  std::vector<int64_t> cnt(counts, counts + C);
  GV_TRY(sphere_project(model, KX, cnt, model->mu, st));
  model->iters = 0;
  return GV_OK;
}

}  // namespace gv
